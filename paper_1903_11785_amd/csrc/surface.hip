// Crossing-edge compaction and exit-point bisection (Sec. II-C) for gfx950.
//
// Crossing edges come from the fine bitmap of each lattice (each x-row padded
// to whole 64-bit words; in a frame the fine carve writes it): one thread per
// word tests 64 samples at once, x-edges by XOR with the word shifted by one
// sample, y- and z-edges by XOR with the words one row and one slab further.
// Work items are kEdgeWords consecutive words of one lattice.  A first pass
// counts each item's edges; a second sums the counts of the items before it
// and writes the keys 3*lin+axis in ascending order (a thread's keys are in
// order, and a block scan orders the threads).  Exit points: a group of four
// lanes per edge sharing its cameras; a first pass keeps the cameras that can
// reject some point of the edge at all, and the bisection tests only those,
// two steps per round.
#include "fvv_internal.h"

#include <type_traits>

namespace fvv {

// The single job of fvv_surface, from the kernel arguments.
__global__ void surface_single_kernel(const fvv_job job, fvv_job* __restrict__ dst,
                                      JobPrefix* __restrict__ pre, uint32_t* __restrict__ counts) {
    if (threadIdx.x == 0) {
        dst[0] = job;
        const int64_t words = fine_bitmap_words(job.grid);
        pre[0].tile_off = 0;
        pre[0].bit_off = 0;
        pre[0].item_off = 0;
        pre[1].item_off = (uint32_t)((words + kEdgeWords - 1) / kEdgeWords);
        counts[3] = 1;
    }
}

// Fine bitmap of one lattice from its uint8 occupancy: one wave per word,
// lane = bit.
__global__ __launch_bounds__(kBlock) void fine_bitmap_kernel(const uint8_t* __restrict__ occ,
                                                             int32_t nx, int32_t wr,
                                                             int64_t n_words,
                                                             uint64_t* __restrict__ bits) {
    const int64_t word = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
    if (word >= n_words)
        return;
    const int64_t row = word / wr;
    const int32_t x = (int32_t)(word - row * wr) * kWave + lane_id();
    const uint64_t b = __ballot(x < nx && occ[row * nx + x] != 0);
    if (lane_id() == 0)
        bits[word] = b;
}

SurfaceScratch surface_scratch(fvv_ctx* ctx) {
    return SurfaceScratch{ctx->d_job_single,
                          ctx->d_prefix,
                          ctx->d_counts_single,
                          ctx->d_point_off_single,
                          ctx->d_finebits,
                          ctx->d_item_cnt,
                          ctx->d_word_edges,
                          ctx->d_status,
                          ctx->d_tsils,
                          tiled_sil_words(ctx->lim.max_cams, ctx->lim.max_w, ctx->lim.max_h),
                          ctx->n_cus};
}

hipError_t launch_surface_prepare_single(const SurfaceScratch& sc, const fvv_job& job,
                                         const uint8_t* occ, hipStream_t s) {
    hipLaunchKernelGGL(surface_single_kernel, dim3(1), dim3(64), 0, s, job, sc.job_single, sc.pre,
                       sc.counts_single);
    const int64_t n_words = fine_bitmap_words(job.grid);
    const int64_t blocks = (n_words * kWave + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(fine_bitmap_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, occ,
                       job.grid.dims[0], (job.grid.dims[0] + 63) / 64, n_words, sc.finebits);
    return hipGetLastError();
}

// ------------------------------------------------------------------ crossing edges
// Crossing-edge masks of word w of a fine bitmap of lattice dims d, wr words
// per row: bit b of ex / ey / ez flags the edge from sample x = 64*q + b of
// the word's row along x / y / z (both ends in the lattice, occupancies
// differ).
struct EdgeMasks {
    uint64_t ex, ey, ez;
    uint64_t v;          // the word's samples
};

__device__ __forceinline__ EdgeMasks edge_masks(const uint64_t* __restrict__ bits, int64_t w,
                                                const int32_t* d, int32_t wr) {
    const int64_t row = w / wr;
    const int32_t q = (int32_t)(w - row * wr);
    const int32_t y = (int32_t)(row % d[1]);
    const int32_t z = (int32_t)(row / d[1]);
    const uint64_t tail = (d[0] & 63) ? (1ull << (d[0] & 63)) - 1 : ~0ull;
    const bool last = q == wr - 1;
    const uint64_t in = last ? tail : ~0ull;           // samples of the lattice
    const bool hy = y + 1 < d[1], hz = z + 1 < d[2];
    // the four loads are issued together (absent ones repeat this word)
    const uint64_t v = bits[w] & in;
    const uint64_t nx = last ? 0ull : bits[w + 1] & (q + 1 == wr - 1 ? tail : ~0ull);
    const uint64_t vy = bits[hy ? w + wr : w];
    const uint64_t vz = bits[hz ? w + (int64_t)wr * d[1] : w];
    EdgeMasks m;
    m.v = v;
    m.ex = (v ^ ((v >> 1) | (nx << 63))) & (last ? tail >> 1 : ~0ull);
    m.ey = hy ? (v ^ vy) & in : 0ull;
    m.ez = hz ? (v ^ vz) & in : 0ull;
    return m;
}

__device__ __forceinline__ uint32_t edge_count(const EdgeMasks& m) {
    return (uint32_t)(__popcll(m.ex) + __popcll(m.ey) + __popcll(m.ez));
}

// Per work item: its number of crossing edges.
__global__ __launch_bounds__(kBlock) void edge_count_kernel(const fvv_job* __restrict__ jobs,
                                                            const JobPrefix* __restrict__ pre,
                                                            const uint32_t* __restrict__ n_jobs_p,
                                                            const uint64_t* __restrict__ bits,
                                                            uint32_t* __restrict__ item_cnt) {
    __shared__ uint32_t table[kJobTable];
    __shared__ uint32_t scratch[kBlock / kWave];
    const int nj = (int)*n_jobs_p;
    const ItemJobs ij = load_item_jobs(pre, nj, table);
    // two copies of the loop, with the job table in LDS and without (so that
    // neither reads it through generic pointers)
    auto items_loop = [&](auto in_lds) {
    constexpr bool kLds = decltype(in_lds)::value;
    const uint32_t n_items = item_first<kLds>(table, pre, nj);
    for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int jb = item_job<kLds>(table, pre, nj, item);
        const fvv_grid g = jobs[jb].grid;
        const int64_t n_words = fine_bitmap_words(g);
        const int64_t w =
            (int64_t)(item - item_first<kLds>(table, pre, jb)) * kEdgeWords + threadIdx.x;
        const int32_t wr = (g.dims[0] + 63) / 64;
        uint32_t c = 0;
        if (w < n_words)
            c = edge_count(edge_masks(bits + pre[jb].bit_off, w, g.dims, wr));
        uint32_t total;
        block_exclusive_sum<kBlock>(c, scratch, &total);
        if (threadIdx.x == 0)
            item_cnt[item] = total;
    }
    };
    if (ij.lds)
        items_loop(std::true_type{});
    else
        items_loop(std::false_type{});
}

// Per work item: first edge = sum of the counts of the items before it; then
// every thread writes its word's keys.  The first item of a job gives the
// job's point offset, the last item the total (ECAPACITY past max_points).
// xyz[3e] carries, until the bisection overwrites it, +1 if the edge's first
// sample (lin of its key) is occupied and -1 otherwise.  kKeys: write the keys,
// xyz marks, offsets and total; kWords: write every word's WordEdges (at the
// job's bit_off, like the bitmap).
template <bool kKeys, bool kWords>
__global__ __launch_bounds__(kBlock) void edge_write_kernel(const fvv_job* __restrict__ jobs,
                                                            const JobPrefix* __restrict__ pre,
                                                            const uint32_t* __restrict__ n_jobs_p,
                                                            const uint64_t* __restrict__ bits,
                                                            const uint32_t* __restrict__ item_cnt,
                                                            uint32_t* __restrict__ keys,
                                                            float* __restrict__ xyz,
                                                            uint32_t max_points,
                                                            uint32_t* __restrict__ point_off,
                                                            uint32_t* __restrict__ n_points,
                                                            WordEdges* __restrict__ wedges,
                                                            uint32_t* __restrict__ status) {
    __shared__ uint32_t table[kJobTable];
    __shared__ uint32_t scratch[kBlock / kWave];
    __shared__ uint64_t scratch64[kBlock / kWave];
    const int nj = (int)*n_jobs_p;
    const ItemJobs ij = load_item_jobs(pre, nj, table);
    // two copies of the loop, with the job table in LDS and without (so that
    // neither reads it through generic pointers)
    auto items_loop = [&](auto in_lds) {
    constexpr bool kLds = decltype(in_lds)::value;
    const uint32_t n_items = item_first<kLds>(table, pre, nj);
    if (kKeys && n_items == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
        for (int j = 0; j <= nj; ++j)
            point_off[j] = 0;
        *n_points = 0;
    }
    for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        // edges of all earlier items
        uint64_t before = 0;
        for (uint32_t i = threadIdx.x; i < item; i += kBlock)
            before += item_cnt[i];
        uint64_t first;
        block_exclusive_sum64<kBlock>(before, scratch64, &first);
        const int jb = item_job<kLds>(table, pre, nj, item);
        const fvv_grid g = jobs[jb].grid;
        const int64_t n_words = fine_bitmap_words(g);
        const int64_t w =
            (int64_t)(item - item_first<kLds>(table, pre, jb)) * kEdgeWords + threadIdx.x;
        const int32_t wr = (g.dims[0] + 63) / 64;
        EdgeMasks m{0ull, 0ull, 0ull, 0ull};
        if (w < n_words)
            m = edge_masks(bits + pre[jb].bit_off, w, g.dims, wr);
        uint32_t total;
        const uint32_t ex = block_exclusive_sum<kBlock>(edge_count(m), scratch, &total);
        uint64_t pos = first + ex;
        if (kWords && w < n_words) {
            WordEdges we;
            we.ex = m.ex;
            we.ey = m.ey;
            we.ez = m.ez;
            we.first = (uint32_t)(pos < 0xffffffffull ? pos : 0xffffffffull);
            we.pad = 0;
            wedges[pre[jb].bit_off + w] = we;
        }
        if (kKeys && w < n_words) {
            const int64_t row = w / wr;
            const uint32_t lin0 =
                (uint32_t)(row * g.dims[0] + (w - row * wr) * kWave);   // sample of bit 0
            for (uint64_t b = m.ex | m.ey | m.ez; b; b &= b - 1) {
                const int bit = __ffsll((unsigned long long)b) - 1;
                const uint32_t key = 3u * (lin0 + (uint32_t)bit);
                const float d = ((m.v >> bit) & 1u) ? 1.0f : -1.0f;
#pragma unroll
                for (int axis = 0; axis < 3; ++axis) {
                    const uint64_t mk = axis == 0 ? m.ex : axis == 1 ? m.ey : m.ez;
                    if ((mk >> bit) & 1u) {
                        if (pos < max_points) {
                            keys[pos] = key + (uint32_t)axis;
                            xyz[3 * pos] = d;
                        }
                        ++pos;
                    }
                }
            }
        }
        if (kKeys && threadIdx.x == 0) {
            const auto clamp = [](uint64_t v) { return (uint32_t)(v < 0xffffffffull ? v : 0xffffffffull); };
            if (item == item_first<kLds>(table, pre, jb))
                point_off[jb] = clamp(first);
            if (item + 1 == n_items) {
                const uint64_t all = first + total;
                point_off[nj] = clamp(all);
                *n_points = clamp(all);
                if (all > max_points)
                    atomicOr(status, kFlagCapacity);
            }
        }
    }
    };
    if (ij.lds)
        items_loop(std::true_type{});
    else
        items_loop(std::false_type{});
}

// ------------------------------------------------------------------ exit points
// Exit points by bisection of the edge parameter against the occupancy test
// (the AND over all cameras).
//
// A camera whose padded pixel rectangle around the whole edge lies inside the
// image and is all foreground accepts every point of the edge: the projection
// of a segment is the segment between its ends' projections, and the rounding
// pad bounds the distance between the real quotient of any point of the
// lattice's box and the rounded quotient the occupancy test floors (the ends'
// quotients here come from rcp, whose error the pad also covers).  Such a
// camera is left out of the edge's bisection.
//
// A workgroup takes 64 edges at a time.  Its first wave decodes them (one
// per lane) into LDS records.  The cull then spreads the (edge, camera) pairs
// over the four waves: wave v takes cameras v, v + 4, ... (each camera's
// matrix uniform, in scalar registers), lane = edge, kCullUnroll cameras'
// loads in flight together, so each wave works through a quarter of the rig.
// A pair's padded rectangle of at most 8 x 8 pixels inside the image gets the
// rectangle's pixels as one 64-bit window (bit 8 r + c = pixel (x0 + c,
// y0 + r) from its top-left corner), built from the 2 x 2 blocks of the tiled
// silhouettes around it: the camera is dropped when the rectangle is all
// foreground, else the pair is appended to the workgroup's LDS list with its
// window.  Cameras with larger rectangles are listed without a window.
// The bisection then runs over the kept pairs, 256 at a time: a pair's lane
// tests its camera at the round's points and ORs the failing points into the
// edge's LDS word; the first wave then advances each edge's bracket.  Every
// tested point's pixel lies in its pair's rectangle, so a pair with a window
// reads the pixel from it: the rounds make no memory access but LDS, except
// for pairs without a window (which load the packed row word, as the plain
// test).  Without tiled silhouettes (tiles NULL) every candidate is kept
// without a window.  The n_steps bisection steps run two at a time: a round
// tests the three points lo + (1, 2, 3) w/4 of the bracket [lo, lo + w] and
// replays the two binary steps from them -- the first step tests the midpoint
// (2), the second the midpoint of the half it kept (3 if 2 was inside, else
// 1) -- so the final bracket is exactly that of n_steps binary steps (all
// points are dyadic, exact in float).  The bracket width w is the same for
// every edge.
constexpr int kBisectJobs = 64;    // jobs whose lattices a workgroup keeps in LDS
constexpr int kBisectEdges = 64;   // edges per workgroup pass (64 or 128)
constexpr int kHalves = kBisectEdges / kWave;   // waves that own edges
static_assert(kHalves >= 1 && kHalves <= kBlock / kWave, "edges per pass");
constexpr int kWinCap = 512;       // kept pairs per workgroup pass with an LDS window
constexpr int kCullUnroll = 2;     // cull cameras whose loads are in flight together
constexpr uint32_t kNoWindow = 0xffffffffu;

// An edge as the passes need it: its first sample's coordinates (the sample
// of its key), the axis coordinate of its second sample, the axis, the ON
// end's index along it (as float), the direction toward the OFF end, the
// lattice spacing and origin on that axis, and the bracket start.
struct EdgeRec {
    float c[3];
    float x1;
    float gq, d, h, o, lo;
    int axis;
    int pad_[2];
};

// The padded pixel rectangle of camera P (rounding pad `pad`) around the
// segment X0-X1: window origin and size when it lies inside the image and
// spans at most 8 x 8 pixels (`small`), else small = false.
struct EdgeRect {
    int x0, y0, nx, ny;   // top-left pixel, columns - 1, rows - 1
    bool small;
};

__device__ __forceinline__ EdgeRect edge_rect(const float* P, float pad, int W, int H,
                                              const float* X0, const float* X1) {
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
    EdgeRect r;
    r.small = front && pad < 1.0f && fx0 >= 0.0f && fy0 >= 0.0f && fx1 < (float)W &&
              fy1 < (float)H && fx1 - fx0 <= 7.0f && fy1 - fy0 <= 7.0f;
    r.x0 = r.small ? (int)fx0 : 0;
    r.y0 = r.small ? (int)fy0 : 0;
    r.nx = r.small ? (int)fx1 - r.x0 : 0;
    r.ny = r.small ? (int)fy1 - r.y0 : 0;
    return r;
}

// The window of rectangle r from the four tiled blocks around its corner
// (b[0] = block (x0/8, y0/8), b[1] the next along x, b[2] the next along y,
// b[3] both; absent ones 0): rows shifted up by y0 % 8, then each row's
// pixels right by x0 % 8 with the next block's pixels shifted in.
__device__ __forceinline__ uint64_t edge_window(const EdgeRect& r, const uint64_t* b) {
    const int ox = r.x0 & 7, oy = 8 * (r.y0 & 7);
    const uint64_t t0 = oy ? (b[0] >> oy) | (b[2] << (64 - oy)) : b[0];
    const uint64_t t1 = oy ? (b[1] >> oy) | (b[3] << (64 - oy)) : b[1];
    const uint64_t lo = (uint64_t)(0xffu >> ox) * 0x0101010101010101ull;
    return ((t0 >> ox) & lo) | ((t1 << ((8 - ox) & 7)) & ~lo & (ox ? ~0ull : 0ull));
}

// Pixel of camera P for the point X (the occupancy test up to the silhouette
// word): px, py and whether w > 0 and the pixel lies in the W x H image.
__device__ __forceinline__ bool point_pixel(const float* P, float X, float Y, float Z, int W,
                                            int H, int& px, int& py) {
    const float a = __builtin_fmaf(P[2], Z, __builtin_fmaf(P[1], Y, __builtin_fmaf(P[0], X, P[3])));
    const float b = __builtin_fmaf(P[6], Z, __builtin_fmaf(P[5], Y, __builtin_fmaf(P[4], X, P[7])));
    const float w = __builtin_fmaf(P[10], Z, __builtin_fmaf(P[9], Y, __builtin_fmaf(P[8], X, P[11])));
    const float r = __builtin_amdgcn_rcpf(w);
    float qa = a * r, qb = b * r;
    const bool tiny = w > 0.0f && w < 0x1p-64f;
    if (__builtin_expect(__ballot(tiny) != 0, 0)) {
        if (tiny) {
            qa = a / w;
            qb = b / w;
        }
    }
    qa = __builtin_amdgcn_fmed3f(qa, -4.0f, (float)W + 4.0f);
    qb = __builtin_amdgcn_fmed3f(qb, -4.0f, (float)H + 4.0f);
    px = exact_floor(a, w, qa);
    py = exact_floor(b, w, qb);
    return (w > 0.0f) & ((unsigned)px < (unsigned)W) & ((unsigned)py < (unsigned)H);
}

template <int kCamsCap>
__global__ __launch_bounds__(kBlock) void bisect_kernel(const fvv_job* __restrict__ jobs,
                                                     const uint32_t* __restrict__ n_jobs_p,
                                                     const uint32_t* __restrict__ point_off,
                                                     const CamSet cams,
                                                     const uint32_t* __restrict__ sils,
                                                     const uint64_t* __restrict__ tiles,
                                                     int n_steps,
                                                     const uint32_t* __restrict__ keys,
                                                     float* __restrict__ xyz,
                                                     uint32_t max_points, int job_lds) {
    constexpr int kWaves = kBlock / kWave;
    __shared__ uint32_t s_off[kBisectJobs + 1];
    __shared__ fvv_grid s_grid[kBisectJobs];
    __shared__ float s_P[kCamsCap][13];              // P, then the rounding pad
    __shared__ EdgeRec s_rec[kBisectEdges];
    __shared__ uint16_t s_pair[kBisectEdges * kCamsCap];   // kept (edge, camera) pairs
    __shared__ uint64_t s_win[kWinCap];
    __shared__ uint32_t s_worg[kWinCap];
    __shared__ uint32_t s_fail[kBisectEdges];
    __shared__ uint32_t s_npairs;
    // the point offsets and lattices of the first job_lds jobs (every job the
    // tables hold, up to kBisectJobs), loaded without waiting for the job count
    for (int j = threadIdx.x; j <= job_lds; j += kBlock) {
        s_off[j] = point_off[j];
        if (j < job_lds)
            s_grid[j] = jobs[j].grid;
    }
    const int nj = (int)*n_jobs_p;
    const bool lds = nj <= job_lds;
    for (int q = threadIdx.x; q < cams.n * 13; q += kBlock) {
        const int c = q / 13, e = q - 13 * c;
        s_P[c][e] = e < 12 ? cams.P[c][e] : cams.pad[c];
    }
    __syncthreads();
    // the chunks' loop, once with the job tables in LDS and once without (two
    // copies, so that neither reads its tables through generic pointers)
    auto chunks_loop = [&](auto in_lds) {
    uint32_t total;
    if constexpr (decltype(in_lds)::value)
        total = s_off[nj];
    else
        total = point_off[nj];
    const uint32_t E = total < max_points ? total : max_points;
    const int64_t cam_words = (int64_t)cams.H * cams.wpr;
    const int tpr = (cams.W + 7) / 8;
    const int64_t tpc = (int64_t)tpr * ((cams.H + 7) / 8);
    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    // contiguous edge ranges per XCD, in chunks of kBisectEdges edges
    const XcdSlice xs = xcd_slice((E + kBisectEdges - 1) / kBisectEdges);
    for (uint64_t chunk = xs.begin + xs.slot; chunk < xs.end; chunk += xs.stride) {
        // the first kHalves waves own the chunk's edges, 64 each: this lane's
        // edge in a wave that owns some (its record at s_rec[el])
        const int el = (wave < kHalves ? wave : 0) * kWave + lane;
        const uint32_t e = (uint32_t)chunk * kBisectEdges + (uint32_t)el;
        const bool act = e < E;
        // 1. the edges' records, by the waves that own them
        if (wave < kHalves) {
            const uint32_t ee = act ? e : E - 1;
            int jb;
            fvv_grid g;
            if constexpr (decltype(in_lds)::value) {
                jb = upper_job([&](int m) { return (uint64_t)s_off[m]; }, nj, ee);
                g = s_grid[jb];
            } else {
                jb = upper_job([&](int m) { return (uint64_t)point_off[m]; }, nj, ee);
                g = jobs[jb].grid;
            }
            const uint32_t key = keys[ee];
            const uint32_t lin = key / 3u;
            const int axis = (int)(key - 3u * lin);
            const uint32_t i = lin % (uint32_t)g.dims[0];
            const uint32_t r = lin / (uint32_t)g.dims[0];
            const uint32_t j = r % (uint32_t)g.dims[1];
            const uint32_t k = r / (uint32_t)g.dims[1];
            // (selects rather than run-time indices into local arrays, which
            // would put them in scratch memory)
            const int gx = g.lo[0] + (int)i, gy = g.lo[1] + (int)j, gz = g.lo[2] + (int)k;
            const int g_axis = axis == 0 ? gx : (axis == 1 ? gy : gz);
            const bool p_on = xyz[3 * (int64_t)ee] > 0.0f;   // left there by the edge pass
            const float o_axis = axis == 0 ? g.origin[0] : (axis == 1 ? g.origin[1] : g.origin[2]);
            EdgeRec mine;
            mine.c[0] = lattice_coord(gx, g.h, g.origin[0]);
            mine.c[1] = lattice_coord(gy, g.h, g.origin[1]);
            mine.c[2] = lattice_coord(gz, g.h, g.origin[2]);
            mine.x1 = lattice_coord(g_axis + 1, g.h, o_axis);
            mine.gq = (float)(g_axis + (p_on ? 0 : 1));
            mine.d = p_on ? 1.0f : -1.0f;
            mine.h = g.h;
            mine.o = o_axis;
            mine.lo = 0.0f;
            mine.axis = axis;
            mine.pad_[0] = mine.pad_[1] = 0;
            s_rec[el] = mine;
            if (el == 0)
                s_npairs = 0u;
        }
        __syncthreads();
        // 2. cull: lane = edge (the chunk's 64-edge parts in turn), wave v the
        //    cameras v, v + 4, ...
        for (int half = 0; half < kHalves; ++half) {
            const int ec = half * kWave + lane;
            const bool act_c = (uint32_t)chunk * kBisectEdges + (uint32_t)ec < E;
            const EdgeRec& er = s_rec[ec];
            const float X0[3] = {er.c[0], er.c[1], er.c[2]};
            const float X1[3] = {er.axis == 0 ? er.x1 : er.c[0], er.axis == 1 ? er.x1 : er.c[1],
                                 er.axis == 2 ? er.x1 : er.c[2]};
            for (int cb = wave; cb < cams.n; cb += kWaves * kCullUnroll) {
                EdgeRect rr[kCullUnroll];
                uint64_t blk[kCullUnroll][4];
#pragma unroll
                for (int u = 0; u < kCullUnroll; ++u) {
                    const int cc = min(cb + u * kWaves, cams.n - 1);
                    rr[u] = edge_rect(cams.Pc(cc), cams.padc(cc), cams.W, cams.H, X0, X1);
                    rr[u].small = rr[u].small && tiles != nullptr && act_c;
                    const bool sm = rr[u].small;
                    const int bx = rr[u].x0 >> 3, by = rr[u].y0 >> 3;
                    const bool nx = ((rr[u].x0 + rr[u].nx) >> 3) != bx;
                    const bool ny = ((rr[u].y0 + rr[u].ny) >> 3) != by;
                    const uint64_t* tb = tiles + cc * tpc + (int64_t)by * tpr + bx;
                    blk[u][0] = blk[u][1] = blk[u][2] = blk[u][3] = 0ull;
                    if (sm)
                        blk[u][0] = tb[0];
                    if (sm && nx)
                        blk[u][1] = tb[1];
                    if (sm && ny)
                        blk[u][2] = tb[tpr];
                    if (sm && nx && ny)
                        blk[u][3] = tb[tpr + 1];
                }
#pragma unroll
                for (int u = 0; u < kCullUnroll; ++u) {
                    const int cc = cb + u * kWaves;
                    if (cc >= cams.n)
                        break;
                    const uint64_t wv = edge_window(rr[u], blk[u]);
                    const uint64_t cols = (uint64_t)((2u << rr[u].nx) - 1u) * 0x0101010101010101ull;
                    const uint64_t m = cols & (~0ull >> (8 * (7 - rr[u].ny)));
                    const bool keep = act_c && !(rr[u].small && (wv & m) == m);
                    const uint64_t kb = __ballot(keep);
                    if (kb == 0ull)
                        continue;
                    uint32_t base = 0u;
                    if (lane == 0)
                        base = atomicAdd(&s_npairs, (uint32_t)__popcll(kb));
                    base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
                    const uint32_t slot = base + lane_rank(kb);
                    if (keep) {
                        s_pair[slot] = (uint16_t)((ec << 5) | cc);
                        if (slot < (uint32_t)kWinCap) {
                            s_win[slot] = rr[u].small ? wv : 0ull;
                            s_worg[slot] = rr[u].small
                                               ? ((uint32_t)rr[u].x0 | ((uint32_t)rr[u].y0 << 16))
                                               : kNoWindow;
                        }
                    }
                }
            }
        }
        __syncthreads();
        const uint32_t n_pairs = s_npairs;
        // 3. the rounds; the owning waves keep each edge's bracket start
        float lo = 0.0f, w = 1.0f;
        for (int st = 0; st < n_steps; st += 2) {
            const bool two = st + 1 < n_steps;   // uniform
            const float w4 = 0.25f * w;
            if (wave < kHalves)
                s_fail[el] = 0u;
            __syncthreads();
            for (uint32_t base = (uint32_t)wave * kWave; base < n_pairs; base += kBlock) {
                const uint32_t pi = base + (uint32_t)lane;
                const bool live = pi < n_pairs;
                const uint32_t pr = s_pair[live ? pi : 0];
                const int pe = (int)(pr >> 5), ca = (int)(pr & 31u);
                const EdgeRec& er = s_rec[pe];
                const bool cached = pi < (uint32_t)kWinCap;
                const uint32_t org = cached ? s_worg[cached ? pi : 0] : kNoWindow;
                const uint64_t wv = cached ? s_win[cached ? pi : 0] : 0ull;
                const bool has_win = org != kNoWindow;
                const int ox = (int)(org & 0xffffu), oy = (int)(org >> 16);
                const float* P = s_P[ca];
                const uint32_t* sc = sils + ca * cam_words;
                uint32_t fail = 0u;
                int px[3], py[3];
                bool ok[3];
                uint32_t word[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const bool on = two || q == 1;
                    const float t = er.lo + (float)(q + 1) * w4;
                    const float ax = __builtin_fmaf(er.gq + er.d * t, er.h, er.o);
                    const float Xp = er.axis == 0 ? ax : er.c[0];
                    const float Yp = er.axis == 1 ? ax : er.c[1];
                    const float Zp = er.axis == 2 ? ax : er.c[2];
                    ok[q] = false;
                    word[q] = 0u;
                    if (on) {
                        ok[q] = point_pixel(P, Xp, Yp, Zp, cams.W, cams.H, px[q], py[q]);
                        if (live && ok[q] && !has_win)
                            word[q] = sc[py[q] * cams.wpr + (px[q] >> 5)];
                    }
                }
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const bool on = two || q == 1;
                    if (!on)
                        continue;
                    const int sh = (8 * (py[q] - oy) + (px[q] - ox)) & 63;
                    const bool in = ok[q] && (has_win ? ((wv >> sh) & 1ull) != 0ull
                                                      : ((word[q] >> (px[q] & 31)) & 1u) != 0u);
                    fail |= in ? 0u : (1u << q);
                }
                if (live && fail)
                    atomicOr(&s_fail[pe], fail);
            }
            __syncthreads();
            if (wave < kHalves) {
                const uint32_t f = s_fail[el];
                if (two) {
                    const int idx = !(f & 2u) ? (!(f & 4u) ? 3 : 2) : (!(f & 1u) ? 1 : 0);
                    lo = lo + (float)idx * w4;
                } else if (!(f & 2u)) {
                    lo = lo + 2.0f * w4;
                }
                s_rec[el].lo = lo;
            }
            w = two ? w4 : 0.5f * w;   // every wave: the width is the same for all edges
            __syncthreads();
        }
        // 4. the exit point: the final bracket's midpoint
        if (wave < kHalves && act) {
            const EdgeRec& er = s_rec[el];
            const float hi = lo + w;
            const float t = 0.5f * (lo + hi);
            const float q = er.gq + er.d * t;
            const float ax = __builtin_fmaf(q, er.h, er.o);
            xyz[3 * (int64_t)e + 0] = er.axis == 0 ? ax : er.c[0];
            xyz[3 * (int64_t)e + 1] = er.axis == 1 ? ax : er.c[1];
            xyz[3 * (int64_t)e + 2] = er.axis == 2 ? ax : er.c[2];
        }
        __syncthreads();   // the next chunk rewrites the records, pairs and count
    }
    };
    if (lds)
        chunks_loop(std::true_type{});
    else
        chunks_loop(std::false_type{});
}

hipError_t launch_edges(const SurfaceScratch& sc, const fvv_job* jobs, const uint32_t* n_jobs_dev,
                        uint32_t* keys, float* xyz, uint32_t max_points, uint32_t* point_off,
                        uint32_t* n_points, bool keys_out, bool word_edges, hipStream_t s) {
    if ((!keys_out && !word_edges) || (word_edges && !sc.word_edges))
        return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)(sc.n_cus * 8);
    hipLaunchKernelGGL(edge_count_kernel, dim3(blocks), dim3(kBlock), 0, s, jobs, sc.pre,
                       n_jobs_dev, sc.finebits, sc.item_cnt);
    auto kernel = keys_out ? (word_edges ? edge_write_kernel<true, true>
                                         : edge_write_kernel<true, false>)
                           : edge_write_kernel<false, true>;
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(kBlock), 0, s, jobs, sc.pre, n_jobs_dev,
                       sc.finebits, sc.item_cnt, keys, xyz, max_points, point_off, n_points,
                       sc.word_edges, sc.status);
    return hipGetLastError();
}

hipError_t launch_bisect(int n_cus, const fvv_job* jobs, int max_jobs, const uint32_t* n_jobs_dev,
                         const uint32_t* point_off, const CamSet& cams, const uint32_t* sils,
                         const uint64_t* tiles, int n_steps, const uint32_t* keys, float* xyz,
                         uint32_t max_points, hipStream_t s, hipEvent_t k_start,
                         hipEvent_t k_stop) {
    // jobs: max_jobs entries, point_off: max_jobs + 1
    const int job_lds = max_jobs < kBisectJobs ? max_jobs : kBisectJobs;
    if (cams.n <= 16)
        hipExtLaunchKernelGGL(bisect_kernel<16>, dim3(n_cus * 16), dim3(kBlock), 0, s, k_start,
                              k_stop, 0, jobs, n_jobs_dev, point_off, cams, sils, tiles, n_steps,
                              keys, xyz, max_points, job_lds);
    else
        hipExtLaunchKernelGGL(bisect_kernel<FVV_MAX_CAMS>, dim3(n_cus * 16), dim3(kBlock), 0, s,
                              k_start, k_stop, 0, jobs, n_jobs_dev, point_off, cams, sils, tiles,
                              n_steps, keys, xyz, max_points, job_lds);
    return hipGetLastError();
}

}  // namespace fvv
