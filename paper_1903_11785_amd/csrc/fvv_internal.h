// Internal declarations of the gfx950 visual-hull library: device helpers
// shared by the kernels, the context layout and the launch functions each
// kernel file provides to the C ABI layer (api.hip).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fvv.h"

namespace fvv {

constexpr int kWave = 64;
constexpr int kBlock = 256;              // threads per workgroup everywhere
constexpr int kEdgeWords = 256;          // fine-bitmap words per crossing-edge work item
constexpr uint32_t kFlagCapacity = 1u;   // sticky device status bits: an output capacity
constexpr uint32_t kFlagJob = 2u;        // was exceeded; a batched job was out of range
// Work counters of a context: [0] next work item, [1] tiles per item, [2] jobs
// (persistent carve); [kCounterMesh] workgroups of the triangle count done;
// [kCounterBoxes] boxes kept by a frame's two-pass coarse carve.
constexpr int kCounters = 8;
constexpr int kCounterMesh = 4;
constexpr int kCounterBoxes = 5;

// Projections of a camera rig passed by value in the kernel arguments.
// pad[c] bounds, for every point of the lattice box the call works in, how far
// the quotients the occupancy test floors can be from the real projection
// (plus the error of an rcp-based quotient); +inf where no bound holds.
struct CamSet {
    float P[FVV_MAX_CAMS][12];
    float pad[FVV_MAX_CAMS];
    int32_t n, W, H, wpr;
    __device__ const float* Pc(int c) const { return P[c]; }
    __device__ float padc(int c) const { return pad[c]; }
};

// The cameras of one job of a batched carve: a slice of a device camera table
// and the job's rounding pads (as CamSet::pad, over the job's lattice box).
struct JobCams {
    const fvv_camera* cam;
    const float* pads;
    int32_t n, W, H, wpr;
    __device__ const float* Pc(int c) const { return cam[c].P; }
    __device__ float padc(int c) const { return pads[c]; }
};

// World box of the samples of g (its corner samples, rounded as the kernels
// round lattice coordinates).
__host__ __device__ inline void grid_box(const fvv_grid& g, double lo[3], double hi[3]) {
    for (int a = 0; a < 3; ++a) {
        lo[a] = (double)__builtin_fmaf((float)g.lo[a], g.h, g.origin[a]);
        hi[a] = (double)__builtin_fmaf((float)(g.lo[a] + g.dims[a] - 1), g.h, g.origin[a]);
    }
}

// Rounding pad of camera P over the world box [lo, hi] (see CamSet::pad).
// Each projection row is a chain of three fmas, so its rounded value is within
// 3u(1+u)^2 < 4u of S = sum |P_k||X_k| + |P_3| (u = 2^-24); the quotient of the
// rounded rows is then within d = (4u S_ab + M 4u S_w) / (w_min - 4u S_w) of the
// real projection wherever |a/w| <= M, and a quotient formed with rcp adds at
// most M 2^-22.  The pad covers a point's rounded quotient against the rcp
// quotients of two other points: 2d + M 2^-21, plus slack.  Double precision,
// no contraction, so host and device compute the same value.
__host__ __device__ inline float rounding_pad(const float* P, int W, int H, const double lo[3],
                                              const double hi[3]) {
#pragma clang fp contract(off)
    const double u = 0x1p-24;
    double s[3] = {0, 0, 0}, wmin = INFINITY;
    for (int corner = 0; corner < 8; ++corner) {
        const double X[3] = {(corner & 1) ? hi[0] : lo[0], (corner & 2) ? hi[1] : lo[1],
                             (corner & 4) ? hi[2] : lo[2]};
        for (int r = 0; r < 3; ++r) {
            double acc = fabs((double)P[4 * r + 3]);
            for (int k = 0; k < 3; ++k)
                acc += fabs((double)P[4 * r + k]) * fabs(X[k]);
            s[r] = fmax(s[r], acc);
        }
        double w = (double)P[11];
        for (int k = 0; k < 3; ++k)
            w += (double)P[8 + k] * X[k];
        wmin = fmin(wmin, w);
    }
    const double M = 4.0 * (double)(W > H ? W : H);
    const double ew = 4.0 * u * s[2];
    if (!(wmin - ew > 0.0))
        return INFINITY;
    const double d = (4.0 * u * fmax(s[0], s[1]) + M * ew) / (wmin - ew);
    const double pad = 2.0 * d + M * 0x1p-21 + 0x1p-10;
    if (!(pad < 0.25))
        return INFINITY;       // too coarse to be useful
    return (float)pad * (1.0f + 0x1p-20f);
}

// The corners' range of u and v and minimum of w (box_radius's first step,
// shared by the radii of several half-extents over one box).
struct BoxProj {
    double umin, umax, vmin, vmax, wmin;
};

__host__ __device__ inline BoxProj box_projection(const float* P, const double lo[3],
                                                  const double hi[3]) {
#pragma clang fp contract(off)
    BoxProj b{INFINITY, -INFINITY, INFINITY, -INFINITY, INFINITY};
    for (int corner = 0; corner < 8; ++corner) {
        const double X[3] = {(corner & 1) ? hi[0] : lo[0], (corner & 2) ? hi[1] : lo[1],
                             (corner & 4) ? hi[2] : lo[2]};
        double r[3];
        for (int q = 0; q < 3; ++q) {
            r[q] = (double)P[4 * q + 3];
            for (int k = 0; k < 3; ++k)
                r[q] += (double)P[4 * q + k] * X[k];
        }
        b.wmin = fmin(b.wmin, r[2]);
        if (r[2] > 0.0) {
            // (one reciprocal per corner: its rounding is far inside the
            // relative slack box_radius adds)
            const double rw = 1.0 / r[2];
            b.umin = fmin(b.umin, r[0] * rw);
            b.umax = fmax(b.umax, r[0] * rw);
            b.vmin = fmin(b.vmin, r[1] * rw);
            b.vmax = fmax(b.vmax, r[1] * rw);
        }
    }
    return b;
}

// Bounds (pixels, u then v) on how far the real projection of camera P moves
// within a box of half-extents e (world units) around any point of the world
// box [lo, hi] (b: box_projection over it): with d = X - C,
// u(C + d) - u(C) = (A.d - u(C) W.d) / w(C + d), A and W the first three
// entries of P's first and third rows (the second row for v), u(C) within the
// range of u over the box's corners (u is monotone along every segment where
// w > 0) and w at least its minimum over the corners.
// Double precision, no contraction, with a relative slack; INFINITY where w
// is not positive over the box.
__host__ __device__ inline void box_radius(const float* P, const BoxProj& b, const double e[3],
                                           double* ru, double* rv) {
#pragma clang fp contract(off)
    if (!(b.wmin > 0.0)) {
        *ru = INFINITY;
        *rv = INFINITY;
        return;
    }
    double su = 0.0, sv = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double wk = (double)P[8 + k];
        su += e[k] * fmax(fabs((double)P[k] - b.umin * wk), fabs((double)P[k] - b.umax * wk));
        sv += e[k] * fmax(fabs((double)P[4 + k] - b.vmin * wk), fabs((double)P[4 + k] - b.vmax * wk));
    }
    *ru = su / b.wmin * (1.0 + 1e-9) + 1e-9;
    *rv = sv / b.wmin * (1.0 + 1e-9) + 1e-9;
}

// Radii of a frame's ROI lattices per (job, camera), kRhoPer floats each: the
// pixel half-widths of the rectangle around the centre projection of a box of
// 4 x 4 x 4 samples (u, v), then of an edge along axis 0, 1, 2 (u, v each),
// each already widened by the camera's rounding pad and a margin for the
// float arithmetic of the rectangle (see rho_rect); INFINITY where no bound.
constexpr int kRhoPer = 8;

// The float half-width r of a rectangle [floor(c - r), floor(c + r)] around a
// centre quotient c (an rcp quotient, |c| < 2^13 after clamping) that holds
// the floored quotient of every point within the real radius `radius` of the
// centre's real projection: the radius, the rounding pad (which covers the
// error of both quotients against the real projections) and 2^-8 for the
// rounding of c -/+ r; rounded up; INFINITY when either is unbounded.
__host__ __device__ inline float rho_rect(double radius, float pad) {
    if (!(radius < 1e6) || !(pad < 1.0f))
        return INFINITY;
    return (float)(radius + (double)pad + 0x1p-8) * (1.0f + 0x1p-20f);
}

// Tile of the carving kernels: TX*TY == 256 threads, TZ samples per thread.
struct TileShape {
    int tx, ty, tz;
};

// ------------------------------------------------------------------ pixel test
// Floor of the real quotient a/w (w > 0) from an approximation q of it that is
// within 1 of it.  floor(q) is then the exact floor or off by one, and the
// signs of the residuals a - n*w and a - (n+1)*w, which a single fma rounds
// without changing, decide which.  Branch-free.
__device__ __forceinline__ int exact_floor(float a, float w, float q) {
    int n = (int)__builtin_floorf(q);
    const float nf = (float)n;
    const float r0 = __builtin_fmaf(-nf, w, a);
    const float r1 = __builtin_fmaf(-(nf + 1.0f), w, a);
    n -= (r0 < 0.0f) ? 1 : 0;
    n += (r1 >= 0.0f) ? 1 : 0;
    return n;
}

// Occupancy test of one projected sample (a, b, w) in one camera: w > 0 and
// pixel (floor(a/w), floor(b/w)) inside the W x H image and foreground in
// `sil` (this camera's [H][wpr] rows).  The quotients come from rcp(w),
// clamped to [-4, dim + 4] so the floor stays exact inside the image and the
// classification right outside it; a positive w below 2^-64 (where rcp would
// overflow; never met in practice) takes the IEEE division instead, behind a
// wave-uniform branch.
__device__ __forceinline__ bool sil_test(float a, float b, float w,
                                         const uint32_t* __restrict__ sil, int W, int H,
                                         int wpr) {
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
    const int px = exact_floor(a, w, qa);
    const int py = exact_floor(b, w, qb);
    const bool ok = (w > 0.0f) & ((unsigned)px < (unsigned)W) & ((unsigned)py < (unsigned)H);
    const uint32_t word = sil[ok ? py * wpr + (px >> 5) : 0];
    return ok & (((word >> (px & 31)) & 1u) != 0u);
}

// G occupancy tests at once, test q of point (X[q], Y[q], Z[q]) in camera
// P[q] with silhouette sil[q]; bit q of the result is its outcome.  Phased so
// that the G silhouette loads are issued together: all projections first, one
// wave-uniform check for the rare tiny w, then all floors and loads, then the
// bits.  Each test is the single-camera test above, operation for operation.
template <int G>
__device__ __forceinline__ uint32_t multi_inside(const float* const* __restrict__ P,
                                                 const float* X, const float* Y, const float* Z,
                                                 const uint32_t* const* __restrict__ sil, int W,
                                                 int H, int wpr) {
    float a[G], b[G], w[G], qa[G], qb[G];
    bool tiny_any = false;
#pragma unroll
    for (int q = 0; q < G; ++q) {
        const float* p = P[q];
        a[q] = __builtin_fmaf(p[2], Z[q], __builtin_fmaf(p[1], Y[q], __builtin_fmaf(p[0], X[q], p[3])));
        b[q] = __builtin_fmaf(p[6], Z[q], __builtin_fmaf(p[5], Y[q], __builtin_fmaf(p[4], X[q], p[7])));
        w[q] = __builtin_fmaf(p[10], Z[q], __builtin_fmaf(p[9], Y[q], __builtin_fmaf(p[8], X[q], p[11])));
        const float r = __builtin_amdgcn_rcpf(w[q]);
        qa[q] = a[q] * r;
        qb[q] = b[q] * r;
        tiny_any |= w[q] > 0.0f && w[q] < 0x1p-64f;
    }
    if (__builtin_expect(__ballot(tiny_any) != 0, 0)) {
#pragma unroll
        for (int q = 0; q < G; ++q)
            if (w[q] > 0.0f && w[q] < 0x1p-64f) {
                qa[q] = a[q] / w[q];
                qb[q] = b[q] / w[q];
            }
    }
    uint32_t word[G];
    int px[G];
    bool ok[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
        px[q] = exact_floor(a[q], w[q], __builtin_amdgcn_fmed3f(qa[q], -4.0f, (float)W + 4.0f));
        const int py =
            exact_floor(b[q], w[q], __builtin_amdgcn_fmed3f(qb[q], -4.0f, (float)H + 4.0f));
        ok[q] = (w[q] > 0.0f) & ((unsigned)px[q] < (unsigned)W) & ((unsigned)py < (unsigned)H);
        word[q] = sil[q][ok[q] ? py * wpr + (px[q] >> 5) : 0];
    }
    uint32_t in = 0;
#pragma unroll
    for (int q = 0; q < G; ++q)
        in |= (uint32_t)(ok[q] & (((word[q] >> (px[q] & 31)) & 1u) != 0u)) << q;
    return in;
}

// One world point against G cameras (AND of the single-camera tests).
template <int G>
__device__ __forceinline__ bool group_inside(const float* const* __restrict__ P, float X, float Y,
                                             float Z, const uint32_t* const* __restrict__ sil,
                                             int W, int H, int wpr) {
    float Xs[G], Ys[G], Zs[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
        Xs[q] = X;
        Ys[q] = Y;
        Zs[q] = Z;
    }
    return multi_inside<G>(P, Xs, Ys, Zs, sil, W, H, wpr) == (1u << G) - 1u;
}

// World coordinate of global lattice index g on one axis.
__device__ __forceinline__ float lattice_coord(int g, float h, float o) {
    return __builtin_fmaf((float)g, h, o);
}

// Test of one world point against camera P (12 floats).
__device__ __forceinline__ bool seen_inside(const float* __restrict__ P, float X, float Y, float Z,
                                            const uint32_t* __restrict__ sil, int W, int H,
                                            int wpr) {
    const float a = __builtin_fmaf(P[2], Z, __builtin_fmaf(P[1], Y, __builtin_fmaf(P[0], X, P[3])));
    const float b = __builtin_fmaf(P[6], Z, __builtin_fmaf(P[5], Y, __builtin_fmaf(P[4], X, P[7])));
    const float w =
        __builtin_fmaf(P[10], Z, __builtin_fmaf(P[9], Y, __builtin_fmaf(P[8], X, P[11])));
    return sil_test(a, b, w, sil, W, H, wpr);
}

// ------------------------------------------------------------------ wave/block helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanes_below_mask() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Inclusive prefix sum over a wave with DPP lane moves: shifts by 1, 2, 4, 8
// within each row of 16 lanes, then row 15 -> rows 1 and 3 and row 31 -> rows
// 2 and 3 (lanes outside the source range add 0).
template <int kCtrl, int kRowMask, bool kBound>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, kRowMask, 0xf, kBound);
}

__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
    v += dpp_u32<0x111, 0xf, true>(v);    // row_shr:1
    v += dpp_u32<0x112, 0xf, true>(v);    // row_shr:2
    v += dpp_u32<0x114, 0xf, true>(v);    // row_shr:4
    v += dpp_u32<0x118, 0xf, true>(v);    // row_shr:8
    v += dpp_u32<0x142, 0xa, false>(v);   // row_bcast:15
    v += dpp_u32<0x143, 0xc, false>(v);   // row_bcast:31
    return v;
}

// LDS-only ordering between the lanes of one wave (the LDS serves a wave's
// requests in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
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

template <int kCtrl, int kRowMask, bool kBound>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
    const uint32_t lo = dpp_u32<kCtrl, kRowMask, kBound>((uint32_t)v);
    const uint32_t hi = dpp_u32<kCtrl, kRowMask, kBound>((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_inclusive_sum64(uint64_t v) {
    v += dpp_u64<0x111, 0xf, true>(v);
    v += dpp_u64<0x112, 0xf, true>(v);
    v += dpp_u64<0x114, 0xf, true>(v);
    v += dpp_u64<0x118, 0xf, true>(v);
    v += dpp_u64<0x142, 0xa, false>(v);
    v += dpp_u64<0x143, 0xc, false>(v);
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

// Carving tiles of lattice g for a TX x (256/TX) x TZ tile.
__host__ __device__ inline uint64_t tiles_of_grid(const fvv_grid& g, int tx, int tz) {
    const int ty = kBlock / tx;
    return (uint64_t)((g.dims[0] + tx - 1) / tx) * (uint64_t)((g.dims[1] + ty - 1) / ty) *
           (uint64_t)((g.dims[2] + tz - 1) / tz);
}

// Rank of this lane among the set lanes of `mask` below it.
__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Work items a persistent workgroup grabs at a time: about 8 grabs per
// workgroup over the whole launch.
__host__ __device__ inline uint32_t grab_size(uint64_t total_tiles, uint32_t blocks) {
    const uint64_t per = (total_tiles + (uint64_t)blocks * 8 - 1) / ((uint64_t)blocks * 8);
    return (uint32_t)(per < 1 ? 1 : (per > 0xffffffffull ? 0xffffffffull : per));
}

// ------------------------------------------------------------------ labelling input
// Row bitmap of a coarse occupancy, the labelling's input: bit x of row
// r = j + ny*k lies in word r*wr + x/64 (each row padded to whole words, the
// bits past nx clear) and bit r of `rowmask` flags a row with a set bit.  Both
// are all-zero between calls: producers OR bits in, the labels' write pass
// after the labelling clears them.
struct RowBits {
    uint64_t* words;
    uint64_t* rowmask;
    int32_t wr;          // words per row, ceil(nx / 64)
};

// Which 8 x 8-pixel blocks of each camera's silhouette hold a foreground
// pixel: bit bx % 64 of word (c * tph + by) * bw + bx / 64 for block (bx, by),
// tph = ceil(H / 8) block rows of bw = ceil(ceil(W / 8) / 64) words.  The
// packing kernels OR the bits into all-zero words; the two-pass carve's second
// pass zeroes them again.
struct SilAny {
    const uint64_t* bits;
    int32_t bw, tph;
};
inline int32_t sil_any_bw(int W) { return ((W + 7) / 8 + 63) / 64; }
inline int64_t sil_any_words(int n, int W, int H) {
    return (int64_t)n * ((H + 7) / 8) * sil_any_bw(W);
}

// The two-pass carve of a lattice of at least kRejectMinSamples samples: the
// silhouettes' non-empty blocks (zeroed by the second pass), a list of up to
// one entry per box of 8 x 8 x 4 samples and its count (0 before the carve;
// the frame's labelling clears it again), and the CU count for the second
// pass.
struct CarveReject {
    SilAny any;
    uint32_t* list;
    uint32_t* count;
    int n_cus;
};
constexpr uint64_t kRejectMinSamples = (uint64_t)1 << 21;

constexpr int kStatsRow = 8;   // per component: count, lo[3], hi[3], smallest linear index

// ------------------------------------------------------------------ device-side job prefix data
// Per job of a batched carve / surface: first carving tile and first
// crossing-edge work item (exclusive prefix sums over the job table).
struct JobPrefix {
    uint64_t tile_off;   // first tile of the job
    uint64_t bit_off;    // first word of the job's fine bitmap
    uint64_t row_off;    // first tile row (tiles sharing y and z) of the job (batched carve)
    uint32_t item_off;   // first crossing-edge work item of the job
    uint32_t pad;
};

// Fine bitmap of one lattice (a job): its occupancy with each x-row padded to
// whole 64-bit words, rows in raster order (bit x of row j + ny*k in word
// (j + ny*k)*ceil(nx/64) + x/64).  The bits past nx are unspecified.
__host__ __device__ inline int64_t fine_bitmap_words(const fvv_grid& g) {
    return (int64_t)g.dims[1] * g.dims[2] * ((g.dims[0] + 63) / 64);
}

// XCD-aware static partition: the workgroups of a launch go to the 8 XCDs
// round-robin in launch order, so the workgroups b with b % 8 == x share XCD
// x's L2.  Item range [begin, end) belongs to XCD x; its workgroups take
// items begin + slot, begin + slot + stride, ...  The grid must be a multiple
// of 8 workgroups.  Every item is covered exactly once whatever the actual
// placement; only cache locality depends on it.
constexpr int kXcds = 8;

struct XcdSlice {
    uint64_t begin, end;
    uint32_t slot, stride;
};

__device__ __forceinline__ XcdSlice xcd_slice(uint64_t n) {
    const uint32_t x = blockIdx.x % kXcds;
    return XcdSlice{n * x / kXcds, n * (x + 1) / kXcds, blockIdx.x / kXcds, gridDim.x / kXcds};
}

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

// Crossing edges of one fine-bitmap word as the compaction lays them out: the
// masks by axis (bit b flags the edge from sample 64 q + b of the word's row)
// and the key-list position of the word's first edge (clamped to 2^32 - 1).
// An edge's position is then first + the edges of lower bits + the lower axes
// at its own bit.
struct alignas(32) WordEdges {
    uint64_t ex, ey, ez;
    uint32_t first;
    uint32_t pad;
};

// Item offsets of the jobs in LDS (when they fit) for the item -> job search
// of the passes over fine-bitmap words.
constexpr int kJobTable = 1024;

struct ItemJobs {
    const JobPrefix* pre;
    const uint32_t* lds;   // item_off of jobs 0..nj, or nullptr
    int nj;
    __device__ int job_of(uint32_t item) const {
        if (lds)
            return upper_job([&](int m) { return (uint64_t)lds[m]; }, nj, item);
        return upper_job([&](int m) { return (uint64_t)pre[m].item_off; }, nj, item);
    }
    __device__ uint32_t first_item(int j) const { return lds ? lds[j] : pre[j].item_off; }
};

__device__ __forceinline__ ItemJobs load_item_jobs(const JobPrefix* __restrict__ pre, int nj,
                                                   uint32_t* table) {
    const bool fit = nj < kJobTable;
    if (fit)
        for (int j = threadIdx.x; j <= nj; j += kBlock)
            table[j] = pre[j].item_off;
    __syncthreads();
    return ItemJobs{pre, fit ? table : nullptr, nj};
}

// The job of work item `item` and the first work item of job j, from the
// LDS table (kLds: `table` is the workgroup's copy) or from the prefixes.
template <bool kLds>
__device__ __forceinline__ int item_job(const uint32_t* table, const JobPrefix* __restrict__ pre,
                                        int nj, uint32_t item) {
    if constexpr (kLds)
        return upper_job([&](int m) { return (uint64_t)table[m]; }, nj, item);
    else
        return upper_job([&](int m) { return (uint64_t)pre[m].item_off; }, nj, item);
}

template <bool kLds>
__device__ __forceinline__ uint32_t item_first(const uint32_t* table,
                                               const JobPrefix* __restrict__ pre, int j) {
    if constexpr (kLds)
        return table[j];
    else
        return pre[j].item_off;
}

struct MeshTable;

}  // namespace fvv

// ------------------------------------------------------------------ context
struct fvv_ctx {
    fvv_limits lim;
    int device;
    // status and counters
    uint32_t* d_status;          // sticky flags
    uint32_t* d_counter;         // persistent carve: [0] next item, [1] grab size, [2] jobs
    // labelling
    uint64_t* d_rowbits;         // row bitmap of the coarse occupancy (RowBits)
    uint64_t* d_rowmask;         // rows with a set bit
    int32_t* d_rmpre;            // row-mask prefix, listed rows, run starts per row, run
    int32_t* d_rows;             // extents, run rows and the union-find forest over runs:
    int32_t* d_rs;               // the global twins of the labelling workgroup's LDS
    int32_t* d_x0;               // arrays, used when those are too small
    int32_t* d_x1;
    int32_t* d_rrow;
    int32_t* d_runP;
    int32_t* d_stats;            // per component: kStatsRow ints, then one label each
    int32_t* d_sample_label;     // label of every occupied coarse sample
    // batched carve / frame
    fvv::JobPrefix* d_prefix;    // per job (max(max_jobs, max_rois) + 1)
    float* d_job_pad;            // rounding pad per (job, camera) of a batched carve
    double* d_soft_acc;          // soft hull: per camera sum g and sum (R X) x g
    fvv::MeshTable* d_mesh_table;  // marching-cubes configurations (built at creation)
    fvv_job* d_job_single;       // the job of a single-ROI fvv_surface call
    fvv_camera* d_cams;          // camera table of fvv_frame
    uint64_t* d_finebits;        // fine bitmaps of the jobs (bit_cap words)
    uint64_t* d_tsils;           // a frame's silhouettes in 8 x 8-pixel blocks
    uint64_t* d_sany;            // their non-empty blocks (SilAny layout)
    float* d_rho;                // a frame's radii per (job, camera), kRhoPer floats each
    uint32_t* d_item_cnt;        // crossing edges per work item
    fvv::WordEdges* d_word_edges;  // per fine-bitmap word (bit_cap), for the mesh
    uint64_t* d_tri_first;       // first triangle of each work item
    uint32_t* d_point_off_single;
    uint32_t* d_counts_single;
    int64_t item_cap;
    int64_t job_cap;
    int64_t bit_cap;
    int n_cus;
    // side branch of a frame's mesh (off the critical path), default priority
    hipStream_t side;
    hipEvent_t ev_join;            // the mesh branch done
    hipEvent_t ev_fine, ev_edges;  // a frame's mesh branch: fine bitmaps, keys ready
};

namespace fvv {

// What the selection kernel of a frame also builds once the ROIs are known:
// the fine lattice job of every carried ROI (Sec. II-B-3) and the prefixes of
// the batched carve and the surface passes.
struct FrameJobs {
    CamSet cams;
    fvv_grid coarse;
    int64_t hc_um, hf_um;
    float h_fine;
    fvv_job* jobs;
    int64_t max_fine;
    uint32_t* counts;
    int tile_x, tile_z;
    uint32_t blocks;
    int64_t bit_cap;     // words of the fine bitmap scratch
    float* rho;          // per (job, camera) radii (kRhoPer floats), written with the jobs
};

// The coarse labels' write pass of a frame (after the labelling): per sample
// v, labels[v] = the sample's component label (0 when unoccupied or filtered
// out by Eq. (1)) and occ[v] cleared where the label is 0.  carve_blocks: the
// workgroups of the launch that carve; the rest write labels.
struct LabelWrite {
    const int32_t* sample_label;
    uint8_t* occ;
    int32_t* labels;
    int64_t V;
    uint32_t carve_blocks;
    // the labelling's row bitmap (rb_n words) and row mask (rm_n words),
    // cleared by the same pass for the next call
    uint64_t* rb_words;
    int64_t rb_n;
    uint64_t* rowmask;
    int64_t rm_n;
};

// Thread t of nth of the write pass: its share of the bitmap clear.
__device__ __forceinline__ void label_write_clear(const LabelWrite& lw, int64_t t, int64_t nth) {
    for (int64_t w = t; w < lw.rb_n; w += nth)
        lw.rb_words[w] = 0ull;
    for (int64_t w = t; w < lw.rm_n; w += nth)
        lw.rowmask[w] = 0ull;
}

__device__ __forceinline__ void label_write_sample(const LabelWrite& lw, int64_t v) {
    if (lw.occ[v]) {
        const int32_t lab = lw.sample_label[v];
        lw.labels[v] = lab;
        if (lab == 0)
            lw.occ[v] = 0;
    } else {
        lw.labels[v] = 0;
    }
}

// Launchers (each returns hipSuccess or the launch error).
hipError_t launch_pack(int n, int W, int H, const uint8_t* masks, uint32_t* sils, hipStream_t s);
// rej: for lattices of at least kRejectMinSamples samples carved with plain
// (depth 1, 2 or 8) tiles, the two-pass carve that first rejects whole boxes
// from the silhouettes' non-empty blocks (null: one pass; t does not apply to
// the two passes).
hipError_t launch_carve(const CamSet& cams, const uint32_t* sils, const fvv_grid& g,
                        TileShape t, uint8_t* occ, const RowBits* rows, hipStream_t s,
                        const CarveReject* rej = nullptr);
// finebits: NULL, or where each job's fine bitmap goes (at its bit_off).
hipError_t launch_carve_batched(fvv_ctx* ctx, const fvv_job* jobs, uint32_t n_jobs,
                                const fvv_camera* cams, const uint32_t* sils, uint8_t* out,
                                uint64_t* finebits, TileShape t, int blocks, bool jobs_prepared,
                                hipStream_t s);
RowBits row_bits(fvv_ctx* ctx, const fvv_grid& g);
// seeded: the row bitmap is already filled (by the coarse carve of a frame).
// labels == nullptr: stop before the grid pass (launch_label_write does it).
hipError_t launch_label(fvv_ctx* ctx, const fvv_grid& g, uint8_t* occ, int32_t* labels,
                        uint32_t t_np, uint32_t t_nb, fvv_roi* rois, uint32_t max_rois,
                        uint32_t* n_rois, bool seeded, const FrameJobs* frame, hipStream_t s);
// The write pass's arguments for lattice g (carve_blocks 0).
LabelWrite label_write_args(fvv_ctx* ctx, const fvv_grid& g, uint8_t* occ, int32_t* labels);
hipError_t launch_label_write(fvv_ctx* ctx, const fvv_grid& g, uint8_t* occ, int32_t* labels,
                              hipStream_t s);
// Soft hull: one camera as the kernels use it (intrinsics and the perturbed
// pose, formed on the host in double and rounded once), and each camera's left
// Jacobian of SO(3) at its rotation perturbation.
struct SoftCam {
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
};

struct SoftCamSet {
    SoftCam c[FVV_MAX_CAMS];
    int32_t n, W, H;
};

struct SoftJacobians {
    double Jl[FVV_MAX_CAMS][9];
};

// Marching-cubes configurations: triangles per corner pattern (at most 5)
// and their cell edges (4 a + u + 2 v).
struct MeshTable {
    uint8_t count[256];
    uint8_t edge[256][15];
};
void build_mesh_table(MeshTable* t);
// Triangles of one lattice (fvv_mesh): its fine bitmap and word edges, then
// the mesh passes, checking every vertex against keys.
hipError_t launch_mesh(fvv_ctx* ctx, const fvv_grid& g, const uint8_t* occ, const uint32_t* keys,
                       const uint32_t* n_keys, uint32_t max_keys, uint32_t* tris,
                       uint32_t max_tris, uint32_t* n_tris, hipStream_t s);
// The mesh passes over the jobs' fine bitmaps (ctx->d_finebits): triangles
// per work item (needs the bitmaps), then the triangles (needs the word edges
// of the edge compaction).  tri_off: NULL, or per job its first triangle and
// at [n_jobs] the total; n_tris: NULL, or the total.  Vertices are positions
// in the key list; those at or past min(*n_keys, max_keys), or (verify) whose
// key differs, are 0xffffffff and set the capacity flag.  items_hint: the
// number of work items when the host knows it, else 0.
hipError_t launch_mesh_count(fvv_ctx* ctx, const fvv_job* jobs, const uint32_t* n_jobs_dev,
                             int64_t items_hint, hipStream_t s);
hipError_t launch_mesh_write(fvv_ctx* ctx, const fvv_job* jobs, const uint32_t* n_jobs_dev,
                             const uint32_t* keys, const uint32_t* n_keys, uint32_t max_keys,
                             bool verify, uint32_t* tris, uint32_t max_tris, uint32_t* tri_off,
                             uint32_t* n_tris, int64_t items_hint, hipStream_t s);

// The paper's Bresenham isovalue of the first min(*n_keys, max_keys) keys.
hipError_t launch_isovalue(fvv_ctx* ctx, const fvv_grid& g, const uint8_t* occ, const CamSet& cams,
                           const uint32_t* sils, const uint32_t* keys, const uint32_t* n_keys,
                           uint32_t max_keys, float* lambda, float* xyz, hipStream_t s);
// The same for a frame's edges (ROI-major keys, per-job offsets), in place of
// the bisection: xyz gets the points at lambda.
hipError_t launch_isovalue_jobs(fvv_ctx* ctx, const fvv_job* jobs, const uint32_t* n_jobs_dev,
                                const uint32_t* point_off, const CamSet& cams,
                                const uint32_t* sils, const uint32_t* keys, float* xyz,
                                uint32_t max_points, hipStream_t s, hipEvent_t k_start = nullptr,
                                hipEvent_t k_stop = nullptr);

// Depth images (cleared, then the triangles' minimum distances) and the
// triangles' visibility masks.
hipError_t launch_visibility(fvv_ctx* ctx, const CamSet& cams, const float* xyz,
                             const uint32_t* n_vert, uint32_t max_vert, const uint32_t* tris,
                             const uint32_t* n_tris, uint32_t max_tris, float t_v, float* depth,
                             uint32_t* vis, hipStream_t s);

bool make_soft_cams(int n, int W, int H, const fvv_soft_camera* in, SoftCamSet* cs,
                    SoftJacobians* jac);
hipError_t launch_soft_forward(fvv_ctx* ctx, const SoftCamSet& cams, const fvv_grid& g,
                               const float* logits, const float* target, float* occ,
                               double* loss, hipStream_t s);
hipError_t launch_soft_backward(fvv_ctx* ctx, const SoftCamSet& cams, const SoftJacobians& jac,
                                const fvv_grid& g, const float* logits, const float* target,
                                const float* grad_occ, const double* scale, float* grad_logits,
                                double* grad_pose, hipStream_t s);
// Device scratch of the crossing-edge and exit-point passes: a context's
// (surface_scratch) or the static array of the allocation-free entry point.
struct SurfaceScratch {
    fvv_job* job_single;         // the job of a single lattice
    JobPrefix* pre;              // per job (at least 2)
    uint32_t* counts_single;     // [3] = jobs of a single lattice (1)
    uint32_t* point_off_single;  // 2 entries
    uint64_t* finebits;          // fine bitmaps of the jobs
    uint32_t* item_cnt;          // crossing edges per work item
    WordEdges* word_edges;       // per fine-bitmap word (NULL: never written)
    uint32_t* status;            // sticky flags
    uint64_t* tiles;             // silhouettes in 8 x 8-pixel blocks (NULL: none)
    int64_t tile_cap;            // words at `tiles`
    int n_cus;
};
SurfaceScratch surface_scratch(fvv_ctx* ctx);
// Crossing edges of the jobs' fine bitmaps: keys (and xyz's side marks),
// point_off and n_points when `keys_out`; the word edges of every word when
// `word_edges`.
hipError_t launch_edges(const SurfaceScratch& sc, const fvv_job* jobs, const uint32_t* n_jobs_dev,
                        uint32_t* keys, float* xyz, uint32_t max_points, uint32_t* point_off,
                        uint32_t* n_points, bool keys_out, bool word_edges, hipStream_t s);
// Exit points of the listed edges.  tiles: the silhouettes in 8 x 8-pixel
// blocks (launch_tile_sils), or NULL (slower: no pixel windows).
hipError_t launch_bisect(int n_cus, const fvv_job* jobs, int max_jobs, const uint32_t* n_jobs_dev,
                         const uint32_t* point_off, const CamSet& cams, const uint32_t* sils,
                         const uint64_t* tiles, int n_steps, const uint32_t* keys, float* xyz,
                         uint32_t max_points, hipStream_t s, hipEvent_t k_start = nullptr,
                         hipEvent_t k_stop = nullptr);
// The fine carve of a frame (jobs prepared by the labelling): tiles with
// tz == 4 classify cameras per box first (rounding pads of `cams`), others
// take the batched carve.
// k_start, k_stop: NULL, or events that take the kernel's own start and end
// times (hipExtLaunchKernel).
// The labels' write pass (launch_label_write's work) runs in the same launch.
hipError_t launch_carve_frame(fvv_ctx* ctx, const fvv_job* jobs, int max_jobs,
                              const CamSet& cams, const uint32_t* sils, const uint64_t* tiles,
                              uint8_t* out, uint64_t* finebits, TileShape t, int blocks,
                              const fvv_grid& coarse, uint8_t* occ_coarse, int32_t* labels,
                              hipStream_t s, hipEvent_t k_start = nullptr,
                              hipEvent_t k_stop = nullptr);
// The silhouettes in 8 x 8-pixel blocks (tile_sils_kernel's layout), from the
// packed rows; any (may be null): the non-empty blocks ORed into SilAny's
// layout (all-zero before).
hipError_t launch_tile_sils(int n, int W, int H, const uint32_t* sils, uint64_t* tiles,
                            uint64_t* any, hipStream_t s);
// Pack the masks into both forms (packed rows and 8 x 8-pixel blocks) in one
// pass where the width is a multiple of 8, else by the two kernels in turn;
// any as for launch_tile_sils.
hipError_t launch_pack_tiled(int n, int W, int H, const uint8_t* masks, uint32_t* sils,
                             uint64_t* tiles, uint64_t* any, hipStream_t s);
// Words of the tiled silhouettes of n cameras of W x H pixels.
inline int64_t tiled_sil_words(int n, int W, int H) {
    return (int64_t)n * ((W + 7) / 8) * ((H + 7) / 8);
}
// The job table and fine bitmap of a single lattice with occupancy occ.
hipError_t launch_surface_prepare_single(const SurfaceScratch& sc, const fvv_job& job,
                                         const uint8_t* occ, hipStream_t s);

}  // namespace fvv
