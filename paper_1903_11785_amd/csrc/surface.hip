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

hipError_t launch_surface_prepare_single(fvv_ctx* ctx, const fvv_job& job, const uint8_t* occ,
                                         hipStream_t s) {
    hipLaunchKernelGGL(surface_single_kernel, dim3(1), dim3(64), 0, s, job, ctx->d_job_single,
                       ctx->d_prefix, ctx->d_counts_single);
    const int64_t n_words = fine_bitmap_words(job.grid);
    const int64_t blocks = (n_words * kWave + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(fine_bitmap_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, occ,
                       job.grid.dims[0], (job.grid.dims[0] + 63) / 64, n_words, ctx->d_finebits);
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
    const uint32_t n_items = ij.first_item(nj);
    for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int jb = ij.job_of(item);
        const fvv_grid g = jobs[jb].grid;
        const int64_t n_words = fine_bitmap_words(g);
        const int64_t w = (int64_t)(item - ij.first_item(jb)) * kEdgeWords + threadIdx.x;
        const int32_t wr = (g.dims[0] + 63) / 64;
        uint32_t c = 0;
        if (w < n_words)
            c = edge_count(edge_masks(bits + pre[jb].bit_off, w, g.dims, wr));
        uint32_t total;
        block_exclusive_sum<kBlock>(c, scratch, &total);
        if (threadIdx.x == 0)
            item_cnt[item] = total;
    }
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
    const uint32_t n_items = ij.first_item(nj);
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
        const int jb = ij.job_of(item);
        const fvv_grid g = jobs[jb].grid;
        const int64_t n_words = fine_bitmap_words(g);
        const int64_t w = (int64_t)(item - ij.first_item(jb)) * kEdgeWords + threadIdx.x;
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
            if (item == ij.first_item(jb))
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
}

// ------------------------------------------------------------------ exit points

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
    // only the words the rectangle covers are loaded, all of them together
    const uint32_t* r0 = sil + y0 * cams.wpr;
    const uint32_t* r1 = sil + y1 * cams.wpr;
    const bool two_w = w1 != w0, two_r = y1 != y0;
    uint32_t a00 = 0, a01 = 0, a10 = 0, a11 = 0;
    if (small)
        a00 = r0[w0];
    if (small && two_w)
        a01 = r0[w1];
    if (small && two_r)
        a10 = r1[w0];
    if (small && two_w && two_r)
        a11 = r1[w1];
    return small && (a00 & m0) == m0 && (a01 & m1) == m1 && (!two_r || (a10 & m0) == m0) &&
           (!two_r || (a11 & m1) == m1);
}

// One crossing edge per lane.  Each lane decodes its edge and keeps the
// cameras that can reject some point of it (the others accept the whole edge;
// kCullChunk cameras' loads in flight together).  The wave then lists its
// (edge, kept camera) pairs in LDS and runs the bisection over that list in
// passes of 64 pairs, so every lane tests one pair per pass however unevenly
// the kept cameras fall on the edges; a pair's failing points are ORed into
// its edge's LDS word and each lane then advances its own edge.  The n_steps
// bisection steps run two at a time: a round tests the three points
// lo + (1, 2, 3) w/4 of the bracket [lo, lo + w] and replays the two binary
// steps from them -- the first step tests the midpoint (2), the second the
// midpoint of the half it kept (3 if 2 was inside, else 1) -- so the final
// bracket is exactly that of n_steps binary steps (all points are dyadic,
// exact in float).  The bracket width w is the same for every edge.
constexpr int kCullChunk = 4;      // cameras whose culling loads are in flight together
constexpr int kBisectJobs = 64;    // jobs whose lattices a workgroup keeps in LDS

// An edge as the pair passes need it: the ON-end sample's coordinates, the
// axis, the ON end's index along it (as float), the direction toward the OFF
// end, the lattice spacing and origin on that axis, and the bracket start.
struct EdgeRec {
    float c[3];
    float gq, d, h, o, lo;
    int axis;
    int pad_[3];
};

template <int kCamsCap>
__global__ __launch_bounds__(kBlock, 6) void bisect_kernel(const fvv_job* __restrict__ jobs,
                                                        const uint32_t* __restrict__ n_jobs_p,
                                                        const uint32_t* __restrict__ point_off,
                                                        const CamSet cams,
                                                        const uint32_t* __restrict__ sils,
                                                        int n_steps,
                                                        const uint32_t* __restrict__ keys,
                                                        float* __restrict__ xyz,
                                                        uint32_t max_points) {
    constexpr int kWaves = kBlock / kWave;
    __shared__ uint32_t s_off[kBisectJobs + 1];
    __shared__ fvv_grid s_grid[kBisectJobs];
    __shared__ float s_P[kCamsCap][12];
    __shared__ EdgeRec s_rec[kWaves][kWave];
    __shared__ uint16_t s_pair[kWaves][kWave * kCamsCap];
    __shared__ uint32_t s_fail[kWaves][kWave];
    const int nj = (int)*n_jobs_p;
    const bool lds = nj <= kBisectJobs;
    if (lds)
        for (int j = threadIdx.x; j <= nj; j += kBlock) {
            s_off[j] = point_off[j];
            if (j < nj)
                s_grid[j] = jobs[j].grid;
        }
    for (int q = threadIdx.x; q < cams.n * 12; q += kBlock)
        s_P[q / 12][q % 12] = cams.P[q / 12][q % 12];
    __syncthreads();
    const uint32_t total = lds ? s_off[nj] : point_off[nj];
    const uint32_t E = total < max_points ? total : max_points;
    const int64_t cam_words = (int64_t)cams.H * cams.wpr;
    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    EdgeRec* const rec = s_rec[wave];
    uint16_t* const pairs = s_pair[wave];
    uint32_t* const fails = s_fail[wave];
    // contiguous edge ranges per XCD, in chunks of one block's edges
    const XcdSlice xs = xcd_slice((E + kBlock - 1) / kBlock);
    for (uint64_t chunk = xs.begin + xs.slot; chunk < xs.end; chunk += xs.stride) {
        const uint32_t e = (uint32_t)chunk * kBlock + threadIdx.x;
        const bool act = e < E;
        const uint32_t ee = act ? e : E - 1;
        int jb;
        fvv_grid g;
        if (lds) {
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
        // (selects rather than run-time indices into local arrays, which would
        // put them in scratch memory)
        const int gx = g.lo[0] + (int)i, gy = g.lo[1] + (int)j, gz = g.lo[2] + (int)k;
        const int g_axis = axis == 0 ? gx : (axis == 1 ? gy : gz);
        const bool p_on = xyz[3 * (int64_t)ee] > 0.0f;   // left there by the edge pass
        const int g_on = g_axis + (p_on ? 0 : 1);
        const float d = p_on ? 1.0f : -1.0f;
        const float o_axis = axis == 0 ? g.origin[0] : (axis == 1 ? g.origin[1] : g.origin[2]);
        const float c[3] = {lattice_coord(gx, g.h, g.origin[0]), lattice_coord(gy, g.h, g.origin[1]),
                            lattice_coord(gz, g.h, g.origin[2])};
        const float x1a = lattice_coord(g_axis + 1, g.h, o_axis);
        const float X0[3] = {c[0], c[1], c[2]};
        const float X1[3] = {axis == 0 ? x1a : c[0], axis == 1 ? x1a : c[1],
                             axis == 2 ? x1a : c[2]};
        // cull: the cameras whose padded rectangle around the edge is not all
        // foreground stay (the same camera on every lane: scalar loads)
        uint32_t keep = 0;
        for (int cb = 0; cb < cams.n; cb += kCullChunk) {
            bool acc[kCullChunk];
#pragma unroll
            for (int u = 0; u < kCullChunk; ++u) {
                const int cc = min(cb + u, cams.n - 1);
                acc[u] = camera_accepts_edge(cams, cc, sils + cc * cam_words, X0, X1);
            }
#pragma unroll
            for (int u = 0; u < kCullChunk; ++u)
                if (cb + u < cams.n && !acc[u])
                    keep |= 1u << (cb + u);
        }
        if (!act)
            keep = 0;
        // this lane's edge record and its pairs, listed wave-wide
        EdgeRec& mine = rec[lane];
        mine.c[0] = c[0];
        mine.c[1] = c[1];
        mine.c[2] = c[2];
        mine.gq = (float)g_on;
        mine.d = d;
        mine.h = g.h;
        mine.o = o_axis;
        mine.lo = 0.0f;
        mine.axis = axis;
        const uint32_t cnt = (uint32_t)__builtin_popcount(keep);
        const uint32_t incl = wave_inclusive_sum(cnt);
        const uint32_t n_pairs = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
        {
            uint32_t pos = incl - cnt;
            for (uint32_t m = keep; m; m &= m - 1)
                pairs[pos++] = (uint16_t)((lane << 5) | (__ffs(m) - 1));
        }
        float lo = 0.0f, w = 1.0f;
        for (int st = 0; st < n_steps; st += 2) {
            const bool two = st + 1 < n_steps;   // uniform
            const float w4 = 0.25f * w;
            fails[lane] = 0u;
            wave_lds_sync();
            for (uint32_t base = 0; base < n_pairs; base += kWave) {
                const uint32_t pi = base + (uint32_t)lane;
                const bool live = pi < n_pairs;
                const uint32_t pr = pairs[live ? pi : 0];
                const int el = (int)(pr >> 5), ca = (int)(pr & 31u);
                const EdgeRec& er = rec[el];
                float Xp[3], Yp[3], Zp[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const float t = er.lo + (float)(q + 1) * w4;
                    const float ax = __builtin_fmaf(er.gq + er.d * t, er.h, er.o);
                    Xp[q] = er.axis == 0 ? ax : er.c[0];
                    Yp[q] = er.axis == 1 ? ax : er.c[1];
                    Zp[q] = er.axis == 2 ? ax : er.c[2];
                }
                const float* P3[3] = {s_P[ca], s_P[ca], s_P[ca]};
                const uint32_t* sc = sils + ca * cam_words;
                const uint32_t* S3[3] = {sc, sc, sc};
                uint32_t fail;
                if (two)
                    fail = ~multi_inside<3>(P3, Xp, Yp, Zp, S3, cams.W, cams.H, cams.wpr) & 7u;
                else
                    fail = (~multi_inside<1>(P3, Xp + 1, Yp + 1, Zp + 1, S3, cams.W, cams.H,
                                             cams.wpr) & 1u) << 1;
                if (live && fail)
                    atomicOr(&fails[el], fail);
            }
            wave_lds_sync();
            const uint32_t f = fails[lane];
            if (two) {
                const int idx = !(f & 2u) ? (!(f & 4u) ? 3 : 2) : (!(f & 1u) ? 1 : 0);
                lo = lo + (float)idx * w4;
                w = w4;
            } else {
                if (!(f & 2u))
                    lo = lo + 2.0f * w4;
                w = 0.5f * w;
            }
            mine.lo = lo;
            wave_lds_sync();
        }
        if (act) {
            const float hi = lo + w;
            const float t = 0.5f * (lo + hi);
            const float q = (float)g_on + d * t;
            const float ax = __builtin_fmaf(q, g.h, o_axis);
            xyz[3 * (int64_t)e + 0] = axis == 0 ? ax : c[0];
            xyz[3 * (int64_t)e + 1] = axis == 1 ? ax : c[1];
            xyz[3 * (int64_t)e + 2] = axis == 2 ? ax : c[2];
        }
        wave_lds_sync();   // the next chunk rewrites this wave's records and pairs
    }
}

hipError_t launch_edges(fvv_ctx* ctx, const fvv_job* jobs, const uint32_t* n_jobs_dev,
                        uint32_t* keys, float* xyz, uint32_t max_points, uint32_t* point_off,
                        uint32_t* n_points, bool keys_out, bool word_edges, hipStream_t s) {
    if (!keys_out && !word_edges)
        return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)(ctx->n_cus * 8);
    hipLaunchKernelGGL(edge_count_kernel, dim3(blocks), dim3(kBlock), 0, s, jobs, ctx->d_prefix,
                       n_jobs_dev, ctx->d_finebits, ctx->d_item_cnt);
    auto kernel = keys_out ? (word_edges ? edge_write_kernel<true, true>
                                         : edge_write_kernel<true, false>)
                           : edge_write_kernel<false, true>;
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(kBlock), 0, s, jobs, ctx->d_prefix, n_jobs_dev,
                       ctx->d_finebits, ctx->d_item_cnt, keys, xyz, max_points, point_off,
                       n_points, ctx->d_word_edges, ctx->d_status);
    return hipGetLastError();
}

hipError_t launch_bisect(fvv_ctx* ctx, const fvv_job* jobs, const uint32_t* n_jobs_dev,
                         const uint32_t* point_off, const CamSet& cams, const uint32_t* sils,
                         int n_steps, const uint32_t* keys, float* xyz, uint32_t max_points,
                         hipStream_t s) {
    if (cams.n <= 16)
        hipLaunchKernelGGL(bisect_kernel<16>, dim3(ctx->n_cus * 8), dim3(kBlock), 0, s, jobs,
                           n_jobs_dev, point_off, cams, sils, n_steps, keys, xyz, max_points);
    else
        hipLaunchKernelGGL(bisect_kernel<FVV_MAX_CAMS>, dim3(ctx->n_cus * 8), dim3(kBlock), 0, s,
                           jobs, n_jobs_dev, point_off, cams, sils, n_steps, keys, xyz,
                           max_points);
    return hipGetLastError();
}

}  // namespace fvv
