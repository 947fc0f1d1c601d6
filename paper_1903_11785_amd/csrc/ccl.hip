// Connected components of the coarse occupancy, size filter, ROI boxes
// (Sec. II-B-2) and, in a frame, the fine lattice of every ROI (Sec. II-B-3)
// for gfx950.
//
// The coarse hull of a sports scene occupies well under 1 % of the volume and
// its occupied samples come in short runs along x, so the labelling works on
// runs, not samples.  The occupancy reaches it as a row bitmap (RowBits): the
// coarse carve of a frame ORs in the bits of its survivors, fvv_label builds
// it with a grid pass.  One workgroup then
//   1. lists the rows with an occupied sample (bit mask over the rows),
//   2. cuts each such row into maximal runs of set bits, numbered in raster
//      order, so run ids ascend with the linear index of the first sample,
//   3. unites, for every row, each run with the runs of the four earlier
//      neighbouring rows (y-1 of the same z; y-1, y, y+1 of z-1) whose
//      extent, widened by one sample, overlaps it -- exactly the 26-adjacency
//      between runs (a two-pointer merge of the two sorted run lists) --
//      linking the larger run id under the smaller with a CAS,
//   4. flattens the forest and numbers the roots in ascending run id,
//   5. adds every run to its root's count and bounding box (LDS atomics),
//   6. applies the Eq. (1) filter T_np <= N(S) <= T_nb and numbers the kept
//      components 1..K in that order -- ascending smallest linear index,
//      whatever the interleaving of the atomics -- writes the ROI table and
//      every occupied sample's label, and clears the bitmap for the next call,
//   7. in a frame, lays out the fine jobs of the carried ROIs.
// Rows, runs, forest and stats live in LDS while they fit, otherwise the same
// steps run on global scratch.  A grid pass finally writes the labels of all
// samples and the filtered occupancy.
#include "fvv_internal.h"

namespace fvv {

constexpr int kLabelThreads = 1024;
constexpr int kRowCap = 4096;    // listed rows held in LDS
constexpr int kRunCap = 6144;    // runs held in LDS
constexpr int kRootCap = 1024;   // components whose stats are held in LDS
// Adjacent run pairs listed in LDS before the unions (in the stats rows' room;
// run ids below 2^16 pack two to a word).
constexpr int kPairCap = kStatsRow * kRootCap + kRootCap;
static_assert(kRunCap <= 65536, "run ids of the LDS pair list take 16 bits");

// ------------------------------------------------------------------ union-find
// Loads and stores of values other threads change concurrently: relaxed
// atomics, at workgroup scope in LDS (plain ds instructions) and at agent
// scope in the global-scratch twin (past the per-CU cache).
template <bool kLds>
__device__ __forceinline__ int32_t ld(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED,
                             kLds ? __HIP_MEMORY_SCOPE_WORKGROUP : __HIP_MEMORY_SCOPE_AGENT);
}

template <bool kLds>
__device__ __forceinline__ void st(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED,
                       kLds ? __HIP_MEMORY_SCOPE_WORKGROUP : __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x with path halving: each visited node is re-pointed at its
// grandparent.  Links only ever change roots (CAS on a node that is still a
// root), and a re-pointed node still reaches the same root through an
// ancestor, so halving races with neither links nor other finds.
template <bool kLds>
__device__ __forceinline__ int32_t find_root(int32_t* P, int32_t x) {
    for (;;) {
        const int32_t p = ld<kLds>(P + x);
        if (p == x)
            return x;
        const int32_t gp = ld<kLds>(P + p);
        if (gp == p)
            return p;
        st<kLds>(P + x, gp);
        x = gp;
    }
}

// Link the roots of runs a and b: the larger run id under the smaller, with a
// CAS that only succeeds while the node is still a root; retry otherwise.
template <bool kLds>
__device__ __forceinline__ void unite(int32_t* P, int32_t a, int32_t b) {
    for (;;) {
        a = find_root<kLds>(P, a);
        b = find_root<kLds>(P, b);
        if (a == b)
            return;
        if (a < b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        int32_t expect = a;
        if (__hip_atomic_compare_exchange_strong(
                P + a, &expect, b, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                kLds ? __HIP_MEMORY_SCOPE_WORKGROUP : __HIP_MEMORY_SCOPE_AGENT))
            return;
    }
}

// Measurement builds (FVV_LABEL_PHASES defined) record, from thread 0 of the
// labelling workgroup, the real-time clock (100 MHz) at the end of each phase
// of the last labelling into label_phase_stamps: [0] entry, [1] row mask
// counted, [2] rows listed, [3] runs cut, [4] adjacent run pairs listed, [5]
// runs united, [6] forest flattened and roots numbered, [7] stats, filter and
// ROI table, [8] labels written, [9] the fine jobs laid out, [10] their
// radii.
constexpr int kLabelPhases = 11;
#ifdef FVV_LABEL_PHASES
__device__ uint64_t label_phase_stamps[kLabelPhases];
__device__ __forceinline__ void label_stamp(int i) {
    if (threadIdx.x == 0)
        label_phase_stamps[i] = __builtin_amdgcn_s_memrealtime();
}
// A stamp where no barrier ends the phase: the barrier, then the stamp.
__device__ __forceinline__ void label_stamp_sync(int i) {
    __syncthreads();
    label_stamp(i);
}
#else
__device__ __forceinline__ void label_stamp(int) {}
__device__ __forceinline__ void label_stamp_sync(int) {}
#endif

// ------------------------------------------------------------------ fine jobs of a frame
// floor(a / b) for integers a, b held exactly in doubles, |a| < 2^53, b > 0:
// the correctly rounded quotient never rounds up to the next integer n (a
// non-integer a / b lies at least 1 / b below n, more than its rounding error
// |a / b| 2^-53), so its floor is exact.
__device__ __forceinline__ double floor_div_exact(double a, double b) {
    return __builtin_floor(a / b);
}

constexpr int64_t kMaxKeyedSamples = 1431655765;  // 3*lin+axis must fit 32 bits

// Map each ROI to its fine lattice (integer micrometres, one-coarse-cell
// dilation, clamped to the coarse lattice's extent), lay the carried ROIs out
// back to back in the fine occupancy buffer and the fine bitmap scratch (the
// longest prefix that fits both), and build the tile and work-item prefixes of
// the batched carve and the surface passes.  box(t, lo, hi) gives ROI t's
// coarse box.  counts: [0] K, [1] fine samples, [3] ROIs carried.
// The radii of jobs 0 .. n-1 and every camera (FrameJobs::rho), one pair per
// thread.
// grid_of(t) gives job t's lattice; threads first .. NT - 1 share the pairs.
template <int NT, typename GridOf>
__device__ __forceinline__ void fine_job_radii(const FrameJobs& fj, uint32_t n, int first,
                                               GridOf grid_of) {
    const int nc = fj.cams.n;
    for (uint32_t p = threadIdx.x - first; p < n * (uint32_t)nc; p += NT - first) {
        const uint32_t t = p / (uint32_t)nc;
        const int c = (int)(p - t * (uint32_t)nc);
        const fvv_grid g = grid_of(t);
        double lo[3], hi[3];
        grid_box(g, lo, hi);
        const float pad = fj.cams.pad[c];
        float* out = fj.rho + ((int64_t)t * FVV_MAX_CAMS + c) * kRhoPer;
        // half-extents: 1.5 h per axis for a box of 4 samples, 0.5 h along the
        // axis of an edge; plus the rounding of the lattice coordinates
        const double h = (double)g.h;
        double slack = 0.0;
        for (int a = 0; a < 3; ++a)
            slack = fmax(slack, fmax(fabs(lo[a]), fabs(hi[a])));
        slack *= 0x1p-20;
        const double eb[3] = {1.5 * h + slack, 1.5 * h + slack, 1.5 * h + slack};
        const BoxProj bp = box_projection(fj.cams.P[c], lo, hi);
        double ru, rv;
        box_radius(fj.cams.P[c], bp, eb, &ru, &rv);
        out[0] = rho_rect(ru, pad);
        out[1] = rho_rect(rv, pad);
        for (int a = 0; a < 3; ++a) {
            double ee[3] = {slack, slack, slack};
            ee[a] = 0.5 * h + slack;
            box_radius(fj.cams.P[c], bp, ee, &ru, &rv);
            out[2 + 2 * a] = rho_rect(ru, pad);
            out[3 + 2 * a] = rho_rect(rv, pad);
        }
    }
}

template <int NT, typename Box>
__device__ __forceinline__ void build_fine_jobs(const FrameJobs& fj, Box box, uint32_t K_all,
                                                uint32_t max_rois, JobPrefix* __restrict__ pre,
                                                uint32_t* __restrict__ counter,
                                                fvv_camera* __restrict__ dcams,
                                                uint32_t* __restrict__ status) {
    // the device camera table, by the threads past the first wave (which lays
    // out the jobs meanwhile)
    for (int c = (int)threadIdx.x - kWave; c >= 0 && c < fj.cams.n; c += NT - kWave) {
        fvv_camera cam;
        for (int e = 0; e < 12; ++e)
            cam.P[e] = fj.cams.P[c][e];
        cam.width = fj.cams.W;
        cam.height = fj.cams.H;
        dcams[c] = cam;
    }
    const uint32_t K = K_all < max_rois ? K_all : max_rois;
    // spacings and coarse indices are integers whose products stay below 2^52
    // (the frame's argument checks), exact in doubles
    const double hc = (double)fj.hc_um, hf = (double)fj.hf_um;
    auto fine_lattice = [&](uint32_t t, fvv_grid& fg) -> int64_t {
        int32_t lo[3], hi[3];
        box(t, lo, hi);
        int64_t V = 1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double c0 = (double)fj.coarse.lo[a];
            const double A = c0 + (double)(lo[a] - 1);
            const double B = c0 + (double)(hi[a] + 1);
            double f0 = floor_div_exact(A * hc, hf);
            double f1 = -floor_div_exact(-B * hc, hf);
            const double fmin = -floor_div_exact(-c0 * hc, hf);
            const double fmax = floor_div_exact((c0 + (double)(fj.coarse.dims[a] - 1)) * hc, hf);
            f0 = f0 < fmin ? fmin : f0;
            f1 = f1 > fmax ? fmax : f1;
            fg.origin[a] = fj.coarse.origin[a];
            fg.lo[a] = (int32_t)f0;
            fg.dims[a] = (int32_t)(f1 - f0 + 1.0);
            V *= (int64_t)fg.dims[a];
        }
        fg.h = fj.h_fine;
        return V;
    };
    auto write_job = [&](uint32_t t, const fvv_grid& fg, uint64_t off) {
        fvv_job j;
        j.grid = fg;
        j.cam_base = 0;
        j.n_cams = fj.cams.n;
        j.width = fj.cams.W;
        j.height = fj.cams.H;
        j.sil_base = 0;
        j.out_offset = (int64_t)off;
        fj.jobs[t] = j;
    };
    auto finish = [&](uint32_t n, uint64_t vox, uint64_t tiles, uint64_t items) {
        pre[n].tile_off = tiles;
        pre[n].item_off = (uint32_t)items;
        fj.counts[0] = K_all;
        fj.counts[1] = (uint32_t)(vox > 0xffffffffull ? 0xffffffffull : vox);
        fj.counts[3] = n;
        counter[0] = 0;
        counter[1] = grab_size(tiles, fj.blocks);
        counter[2] = n;
        counter[kCounterBoxes] = 0;   // for the next frame's two-pass coarse carve
        if (n < K_all)
            atomicOr(status, kFlagCapacity);
    };
    // the layout in the first wave, 64 ROIs at a time with wave scans and no
    // workgroup barrier, and meanwhile the radii of every ROI's fine lattice
    // by the other threads (those of ROIs past the carried ones are computed
    // too and never read)
    if (threadIdx.x >= kWave) {
        fine_job_radii<NT>(fj, K, kWave, [&](uint32_t t) {
            fvv_grid fg{};
            fine_lattice(t, fg);
            return fg;
        });
        return;
    }
    auto lane64 = [](uint64_t v, int l) {
        return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l) << 32) |
               (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    };
    // running totals over the chunks before (wave-uniform)
    uint64_t c_vox = 0, c_bits = 0, c_tiles = 0, c_items = 0;
    uint32_t n = K;
    for (uint32_t base = 0; base < K; base += kWave) {
        const uint32_t t = base + threadIdx.x;
        fvv_grid fg{};
        const int64_t V = t < K ? fine_lattice(t, fg) : 0;
        const uint64_t words = t < K ? (uint64_t)fine_bitmap_words(fg) : 0;
        const uint64_t inc_v = wave_inclusive_sum64((uint64_t)V);
        const uint64_t inc_b = wave_inclusive_sum64(words);
        const uint64_t off = c_vox + inc_v - (uint64_t)V, boff = c_bits + inc_b - words;
        // the carried ROIs are the prefix before the first one that does not fit
        const bool bad = t < K && (off + (uint64_t)V > (uint64_t)fj.max_fine ||
                                   V > kMaxKeyedSamples || boff + words > (uint64_t)fj.bit_cap);
        const uint64_t bad_lanes = __ballot(bad);
        const uint32_t end = bad_lanes ? base + (uint32_t)(__ffsll((unsigned long long)bad_lanes) - 1)
                                       : (K < base + kWave ? K : base + kWave);
        const bool fits = t < end;
        const uint64_t tiles = fits ? tiles_of_grid(fg, fj.tile_x, fj.tile_z) : 0;
        const uint64_t items = fits ? (words + kEdgeWords - 1) / kEdgeWords : 0;
        const uint64_t inc_t = wave_inclusive_sum64(tiles);
        const uint64_t inc_i = wave_inclusive_sum64(items);
        if (fits) {
            write_job(t, fg, off);
            pre[t].tile_off = c_tiles + inc_t - tiles;
            pre[t].bit_off = boff;
            pre[t].item_off = (uint32_t)(c_items + inc_i - items);
        }
        // lanes past `end` add no tiles or items, and no voxels or words past K
        c_vox += end > base ? lane64(inc_v, (int)(end - base) - 1) : 0;
        c_bits += lane64(inc_b, kWave - 1);
        c_tiles += lane64(inc_t, kWave - 1);
        c_items += lane64(inc_i, kWave - 1);
        if (bad_lanes) {
            n = end;
            break;
        }
    }
    if (threadIdx.x == 0)
        finish(n, c_vox, c_tiles, c_items);
    label_stamp(9);
}

// ------------------------------------------------------------------ run labelling
constexpr int kMaskCap = 1024;   // row-mask words held in LDS (grids of up to 65536 rows)
constexpr int kRowWords = 4;     // row-bitmap words a thread keeps in registers

// Rows, runs and forest: LDS arrays or their global-scratch twins.
struct RunArrays {
    uint64_t* rm;      // row-mask words
    int32_t* rmpre;    // listed rows before each row-mask word
    int32_t* rows;     // listed rows, ascending
    int32_t* rs;       // first run of each listed row, rs[n_rows] = runs; once the
                       // runs are united, the component rank of each label
    int32_t* x0;       // run extents (global twin) ...
    int32_t* x1;
    uint32_t* xx;      // ... or packed x0 | x1 << 16 (LDS)
    int32_t* rrow;     // row (y + ny z) of each run
    int32_t* P;        // union-find parent; after ranking, -1 - rank at roots
};

struct LabelArgs {
    RowBits rb;
    int32_t nx, ny, nz;
    RunArrays g;                 // global scratch (used when LDS is too small)
    int32_t* gstats;             // global stats rows, kStatsRow per component, then labels
    int32_t* sample_label;       // label of every occupied sample (for the grid pass)
    uint32_t t_np, t_nb;
    fvv_roi* rois;
    uint32_t max_rois;
    uint32_t* n_rois;
    uint32_t* status;
    JobPrefix* pre;
    uint32_t* counter;
    fvv_camera* dcams;
};

template <bool kLds>
__device__ __forceinline__ void put_run(const RunArrays& m, int32_t k, int32_t x0, int32_t x1) {
    if (kLds) {
        m.xx[k] = (uint32_t)x0 | ((uint32_t)x1 << 16);
    } else {
        m.x0[k] = x0;
        m.x1[k] = x1;
    }
}

template <bool kLds>
__device__ __forceinline__ int2 get_run(const RunArrays& m, int32_t k) {
    if (kLds) {
        const uint32_t v = m.xx[k];
        return make_int2((int32_t)(v & 0xffffu), (int32_t)(v >> 16));
    }
    return make_int2(m.x0[k], m.x1[k]);
}

// List index of row r, or -1 when the row has no occupied sample: the rank of
// its bit in the row mask.
__device__ __forceinline__ int32_t row_index(const RunArrays& m, int32_t r) {
    const uint64_t wv = m.rm[r >> 6];
    const uint64_t bit = 1ull << (r & 63);
    return (wv & bit) ? m.rmpre[r >> 6] + __popcll(wv & (bit - 1)) : -1;
}

// Rank of the component of run k (P flattened and ranked).
template <bool kLds>
__device__ __forceinline__ int32_t rank_of(const int32_t* P, int32_t k) {
    const int32_t p = ld<kLds>(P + k);
    return p < 0 ? -1 - p : -1 - ld<kLds>(P + p);
}

// Row-mask word w with the bits of rows >= R cleared, and word q of a row
// with the bits of x >= nx cleared: producers never set them, and masking
// keeps stale scratch from reaching outside the grid.
__device__ __forceinline__ uint64_t rowmask_word(const RowBits& rb, int32_t w, int32_t R) {
    const uint64_t v = rb.rowmask[w];
    return (w == (R - 1) / 64 && (R & 63)) ? v & ((1ull << (R & 63)) - 1) : v;
}

__device__ __forceinline__ uint64_t row_word(const uint64_t* rw, int32_t q, int32_t wr, int32_t nx) {
    const uint64_t v = rw[q];
    return (q == wr - 1 && (nx & 63)) ? v & ((1ull << (nx & 63)) - 1) : v;
}

// Stats rows: count, lo[3], hi[3], smallest linear index.
constexpr int kStatCount = 0, kStatLo = 1, kStatHi = 4, kStatMin = 7;

template <bool kLdsStats>
__device__ __forceinline__ int32_t stat_load(const int32_t* s) {
    return ld<kLdsStats>(s);
}

// Stats of every component (one set of atomics per run), the Eq. (1) filter
// and the numbering in root order (= ascending smallest linear index), the
// ROI table, and per label its component rank (in m.rs, free by now).
template <bool kLds, bool kLdsStats>
__device__ __forceinline__ void stats_and_select(const LabelArgs& a, const RunArrays& m,
                                                 int32_t n_runs, int32_t K_all, int32_t* stats,
                                                 int32_t* labels_of_rank, int32_t* rank_of_label,
                                                 uint32_t* scan, uint32_t* Kout) {
    constexpr int NT = kLabelThreads;
    for (int32_t j = threadIdx.x; j < K_all; j += NT) {
        int32_t* s = stats + (int64_t)kStatsRow * j;
        s[kStatCount] = 0;
        s[kStatLo + 0] = s[kStatLo + 1] = s[kStatLo + 2] = 0x7fffffff;
        s[kStatHi + 0] = s[kStatHi + 1] = s[kStatHi + 2] = -1;
        s[kStatMin] = 0x7fffffff;
    }
    __syncthreads();
    for (int32_t k = threadIdx.x; k < n_runs; k += NT) {
        const int32_t r = m.rrow[k];
        const int32_t y = r % a.ny, z = r / a.ny;
        const int2 x = get_run<kLds>(m, k);
        int32_t* s = stats + (int64_t)kStatsRow * rank_of<kLds>(m.P, k);
        atomicAdd(&s[kStatCount], x.y - x.x + 1);
        atomicMin(&s[kStatLo + 0], x.x);
        atomicMax(&s[kStatHi + 0], x.y);
        atomicMin(&s[kStatLo + 1], y);
        atomicMax(&s[kStatHi + 1], y);
        atomicMin(&s[kStatLo + 2], z);
        atomicMax(&s[kStatHi + 2], z);
        atomicMin(&s[kStatMin], (int32_t)((int64_t)a.nx * r + x.x));
    }
    __syncthreads();
    uint32_t K = 0;
    for (int32_t base = 0; base < K_all; base += NT) {
        const int32_t j = base + threadIdx.x;
        const int32_t* s = stats + (int64_t)kStatsRow * j;
        uint32_t cnt = 0;
        bool keep = false;
        if (j < K_all) {
            cnt = (uint32_t)stat_load<kLdsStats>(&s[kStatCount]);
            keep = a.t_np <= cnt && cnt <= a.t_nb;
        }
        uint32_t total;
        const uint32_t lab = K + block_exclusive_sum<NT>(keep ? 1u : 0u, scan, &total) + 1;
        if (j < K_all)
            labels_of_rank[j] = keep ? (int32_t)lab : 0;
        if (keep && lab <= a.max_rois) {
            fvv_roi roi;
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                roi.lo[e] = stat_load<kLdsStats>(&s[kStatLo + e]);
                roi.hi[e] = stat_load<kLdsStats>(&s[kStatHi + e]);
            }
            roi.count = cnt;
            roi.min_index = (uint32_t)stat_load<kLdsStats>(&s[kStatMin]);
            a.rois[lab - 1] = roi;
            rank_of_label[lab - 1] = j;
        }
        K += total;
    }
    *Kout = K;
}

// Every run b adjacent to run k in an earlier neighbouring row: (y-1, z) and
// (y-1..y+1, z-1).  A row's runs ascend in x, so the scan of a row stops at
// the first run starting past k's reach.
template <bool kLds, typename F>
__device__ __forceinline__ void for_each_earlier_adjacent(const LabelArgs& a, const RunArrays& m,
                                                          int32_t k, F f) {
    const int32_t r = m.rrow[k];
    const int32_t y = r % a.ny, z = r / a.ny;
    const int2 xk = get_run<kLds>(m, k);
    // the four rows' list indices, their run ranges and their first runs, each
    // step's loads issued together
    int32_t jn[4];
    jn[0] = y > 0 ? row_index(m, r - 1) : -1;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int32_t yy = y - 1 + d;
        jn[1 + d] = (z > 0 && yy >= 0 && yy < a.ny) ? row_index(m, r - a.ny - 1 + d) : -1;
    }
    int32_t b[4], be[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        b[q] = jn[q] >= 0 ? m.rs[jn[q]] : 0;
        be[q] = jn[q] >= 0 ? m.rs[jn[q] + 1] : 0;
    }
    int2 xb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        xb[q] = b[q] < be[q] ? get_run<kLds>(m, b[q]) : make_int2(0, 0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        while (b[q] < be[q] && xb[q].x <= xk.y + 1) {
            if (xb[q].y + 1 >= xk.x)
                f(b[q]);
            if (++b[q] < be[q])
                xb[q] = get_run<kLds>(m, b[q]);
        }
    }
}

// The labelling with rows, runs and forest in `m`.  With kLds, gives up
// (returns false, before any global state changed) when the runs do not fit
// the LDS arrays.
template <bool kLds, bool kJobs>
__device__ __forceinline__ bool label_body(const LabelArgs& a, const FrameJobs& fj,
                                           const RunArrays& m, int32_t n_rows,
                                           int32_t* lds_stats, uint32_t* scan) {
    constexpr int NT = kLabelThreads;
    const int32_t R = a.ny * a.nz;
    const int32_t n_rm = (R + 63) / 64;
    const int32_t wr = a.rb.wr;
    // 1. listed rows, ascending (the LDS row mask and its prefix are ready;
    //    the global twin builds the prefix here)
    int32_t pos0 = 0;
    for (int32_t base = 0; base < n_rm; base += NT) {
        const int32_t w = base + threadIdx.x;
        uint64_t bits;
        int32_t pos;
        if (kLds) {
            bits = w < n_rm ? m.rm[w] : 0ull;
            pos = w < n_rm ? m.rmpre[w] : 0;
        } else {
            bits = w < n_rm ? rowmask_word(a.rb, w, R) : 0ull;
            uint32_t total;
            pos = pos0 + (int32_t)block_exclusive_sum<NT>((uint32_t)__popcll(bits), scan, &total);
            if (w < n_rm)
                m.rmpre[w] = pos;
            pos0 += (int32_t)total;
        }
        for (uint64_t b = bits; b; b &= b - 1)
            m.rows[pos++] = w * 64 + (__ffsll((unsigned long long)b) - 1);
    }
    __syncthreads();
    label_stamp(2);
    // 2. runs of each row, numbered in raster order: a run starts at a set
    //    bit whose left neighbour is clear and ends at one whose right
    //    neighbour is clear
    int32_t n_runs = 0;
    for (int32_t base = 0; base < n_rows; base += NT) {
        const int32_t i = base + threadIdx.x;
        const bool act = i < n_rows;
        const int32_t r_i = act ? m.rows[i] : 0;
        const uint64_t* rw = a.rb.words + (int64_t)r_i * wr;
        uint64_t cw[kRowWords + 1];
#pragma unroll
        for (int q = 0; q <= kRowWords; ++q)
            cw[q] = act && q < wr ? row_word(rw, q, wr, a.nx) : 0ull;
        uint32_t cnt = 0;
        uint64_t carry = 0;
#pragma unroll
        for (int q = 0; q < kRowWords; ++q) {
            cnt += (uint32_t)__popcll(cw[q] & ~((cw[q] << 1) | carry));
            carry = cw[q] >> 63;
        }
        if (act)
            for (int32_t q = kRowWords; q < wr; ++q) {
                const uint64_t v = row_word(rw, q, wr, a.nx);
                cnt += (uint32_t)__popcll(v & ~((v << 1) | carry));
                carry = v >> 63;
            }
        uint32_t total;
        const int32_t first = n_runs + (int32_t)block_exclusive_sum<NT>(cnt, scan, &total);
        if (kLds && n_runs + (int32_t)total > kRunCap)
            return false;
        if (act) {
            m.rs[i] = first;
            int32_t k = first, x_start = 0;
            auto emit = [&](int32_t q, uint64_t v, uint64_t nxt, uint64_t cin) {
                const uint64_t st = v & ~((v << 1) | cin);
                const uint64_t en = v & ~((v >> 1) | (nxt << 63));
                for (uint64_t b = st | en; b; b &= b - 1) {
                    const int bit = __ffsll((unsigned long long)b) - 1;
                    const int32_t x = q * 64 + bit;
                    if ((st >> bit) & 1u)
                        x_start = x;
                    if ((en >> bit) & 1u) {
                        put_run<kLds>(m, k, x_start, x);
                        m.rrow[k] = r_i;
                        m.P[k] = k;
                        ++k;
                    }
                }
            };
            uint64_t cin = 0;
#pragma unroll
            for (int q = 0; q < kRowWords; ++q) {
                emit(q, cw[q], cw[q + 1], cin);
                cin = cw[q] >> 63;
            }
            for (int32_t q = kRowWords; q < wr; ++q) {
                const uint64_t v = row_word(rw, q, wr, a.nx);
                emit(q, v, q + 1 < wr ? row_word(rw, q + 1, wr, a.nx) : 0ull, cin);
                cin = v >> 63;
            }
        }
        n_runs += (int32_t)total;
    }
    if (threadIdx.x == 0)
        m.rs[n_rows] = n_runs;
    __syncthreads();
    label_stamp(3);
    // 3. unite every run with the adjacent runs of its earlier neighbouring rows.
    //    In LDS the adjacent pairs are listed first (in the stats rows, unused
    //    until step 5), then united one pair per thread, so that no wave waits
    //    on the neighbour search of some lanes and the unions of others at
    //    once; pairs past the list's room are united where they are found.
    if (kLds) {
        uint32_t* const pairs = reinterpret_cast<uint32_t*>(lds_stats);
        uint32_t* const n_pairs = scan;            // free until the next scan
        if (threadIdx.x == 0)
            *n_pairs = 0u;
        __syncthreads();
        for (int32_t k = threadIdx.x; k < n_runs; k += NT)
            for_each_earlier_adjacent<kLds>(a, m, k, [&](int32_t b) {
                const uint64_t act = __ballot(true);
                const int leader = __ffsll((unsigned long long)act) - 1;
                uint32_t base = 0;
                if (lane_id() == leader)
                    base = atomicAdd(n_pairs, (uint32_t)__popcll(act));
                const uint32_t slot =
                    (uint32_t)__builtin_amdgcn_readlane((int)base, leader) + lane_rank(act);
                if (slot < (uint32_t)kPairCap)
                    pairs[slot] = ((uint32_t)k << 16) | (uint32_t)b;
                else
                    unite<kLds>(m.P, k, b);
            });
        __syncthreads();
        label_stamp(4);
        const uint32_t np = min(*n_pairs, (uint32_t)kPairCap);
        for (uint32_t q = threadIdx.x; q < np; q += NT) {
            const uint32_t v = pairs[q];
            unite<kLds>(m.P, (int32_t)(v >> 16), (int32_t)(v & 0xffffu));
        }
    } else {
        label_stamp(4);
        for (int32_t k = threadIdx.x; k < n_runs; k += NT)
            for_each_earlier_adjacent<kLds>(a, m, k, [&](int32_t b) { unite<kLds>(m.P, k, b); });
    }
    __syncthreads();
    label_stamp(5);
    // 4. flatten, then number the roots in ascending run id.  The walk only
    //    reads: the sole writes now set a node to its root, which keeps every
    //    concurrent walk on course (path halving here could store a
    //    grandparent over a root written meanwhile).
    for (int32_t k = threadIdx.x; k < n_runs; k += NT) {
        int32_t x = k;
        for (int32_t p = ld<kLds>(m.P + x); p != x; p = ld<kLds>(m.P + x))
            x = p;
        st<kLds>(m.P + k, x);
    }
    __syncthreads();
    int32_t K_all = 0;
    for (int32_t base = 0; base < n_runs; base += NT) {
        const int32_t k = base + threadIdx.x;
        const bool root = k < n_runs && ld<kLds>(m.P + k) == k;
        uint32_t total;
        const uint32_t rk = block_exclusive_sum<NT>(root ? 1u : 0u, scan, &total);
        if (root)
            st<kLds>(m.P + k, -1 - (K_all + (int32_t)rk));
        K_all += (int32_t)total;
    }
    __syncthreads();
    label_stamp(6);
    // 5. stats, filter, ROI table (stats rows in LDS while the components fit;
    //    the label of each rank follows the rows)
    uint32_t K = 0;
    const bool lds_stats_ok = K_all <= kRootCap;
    if (lds_stats_ok)
        stats_and_select<kLds, true>(a, m, n_runs, K_all, lds_stats,
                                     lds_stats + (int64_t)kStatsRow * kRootCap, m.rs, scan, &K);
    else
        stats_and_select<kLds, false>(a, m, n_runs, K_all, a.gstats,
                                      a.gstats + (int64_t)kStatsRow * K_all, a.g.rs, scan, &K);
    __syncthreads();
    label_stamp(7);
    // 6. labels of the occupied samples (the write pass that follows clears the
    //    bitmap for the next call)
    for (int32_t k = threadIdx.x; k < n_runs; k += NT) {
        const int64_t row_lin = (int64_t)a.nx * m.rrow[k];
        const int32_t rk = rank_of<kLds>(m.P, k);
        const int32_t l = lds_stats_ok ? ld<true>(lds_stats + (int64_t)kStatsRow * kRootCap + rk)
                                       : ld<false>(a.gstats + (int64_t)kStatsRow * K_all + rk);
        const int2 x = get_run<kLds>(m, k);
        for (int32_t xi = x.x; xi <= x.y; ++xi)
            a.sample_label[row_lin + xi] = l;
    }
    if (threadIdx.x == 0) {
        *a.n_rois = K;
        if (K > a.max_rois)
            atomicOr(a.status, kFlagCapacity);
    }
    if (kJobs) {
        __syncthreads();
        label_stamp(8);
        auto box = [&](uint32_t t, int32_t* lo, int32_t* hi) {
            if (lds_stats_ok) {
                const int32_t* s = lds_stats + (int64_t)kStatsRow * m.rs[t];
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    lo[e] = ld<true>(&s[kStatLo + e]);
                    hi[e] = ld<true>(&s[kStatHi + e]);
                }
            } else {
                const int32_t* s = a.gstats + (int64_t)kStatsRow * ld<false>(a.g.rs + t);
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    lo[e] = ld<false>(&s[kStatLo + e]);
                    hi[e] = ld<false>(&s[kStatHi + e]);
                }
            }
        };
        build_fine_jobs<NT>(fj, box, K, a.max_rois, a.pre, a.counter, a.dcams, a.status);
        label_stamp_sync(10);
    }
    return true;
}

template <bool kJobs>
__global__ __launch_bounds__(kLabelThreads) void label_runs_kernel(const LabelArgs a,
                                                                   const FrameJobs fj) {
    __shared__ uint64_t s_rm[kMaskCap];
    __shared__ int32_t s_rmpre[kMaskCap];
    __shared__ int32_t s_rows[kRowCap];
    __shared__ int32_t s_rs[kRowCap + 1];
    __shared__ uint32_t s_xx[kRunCap];
    __shared__ int32_t s_rrow[kRunCap];
    __shared__ int32_t s_P[kRunCap];
    __shared__ int32_t s_stats[kStatsRow * kRootCap + kRootCap];   // rows, then labels
    __shared__ uint32_t s_scan[kLabelThreads / kWave];
    label_stamp(0);
    const int32_t R = a.ny * a.nz;
    const int32_t n_rm = (R + 63) / 64;
    const bool lds_ok = n_rm <= kMaskCap && a.nx <= 65535;
    // listed rows: count them, and keep the row mask and its prefix in LDS
    int32_t n_rows = 0;
    for (int32_t base = 0; base < n_rm; base += kLabelThreads) {
        const int32_t w = base + threadIdx.x;
        const uint64_t bits = w < n_rm ? rowmask_word(a.rb, w, R) : 0ull;
        uint32_t total;
        const uint32_t ex =
            block_exclusive_sum<kLabelThreads>((uint32_t)__popcll(bits), s_scan, &total);
        if (lds_ok && w < n_rm) {
            s_rm[w] = bits;
            s_rmpre[w] = n_rows + (int32_t)ex;
        }
        n_rows += (int32_t)total;
    }
    __syncthreads();
    label_stamp(1);
    if (lds_ok && n_rows <= kRowCap) {
        const RunArrays m{s_rm, s_rmpre, s_rows, s_rs, nullptr, nullptr, s_xx, s_rrow, s_P};
        if (label_body<true, kJobs>(a, fj, m, n_rows, s_stats, s_scan))
            return;
        __syncthreads();
    }
    label_body<false, kJobs>(a, fj, a.g, n_rows, s_stats, s_scan);
}

// Row bitmap of an occupancy grid: one wave per (row, word), lane = bit.
// Every word of the grid is stored (zeros included); rows with a set bit are
// ORed into the (all-zero) row mask.
__global__ __launch_bounds__(kBlock) void label_bitmap_kernel(const uint8_t* __restrict__ occ,
                                                              int32_t nx, int64_t n_words,
                                                              const RowBits rb) {
    const int64_t word = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
    if (word >= n_words)
        return;
    const int64_t row = word / rb.wr;
    const int32_t x = (int32_t)(word - row * rb.wr) * kWave + lane_id();
    const bool on = x < nx && occ[row * nx + x] != 0;
    const uint64_t bits = __ballot(on);
    if (lane_id() == 0) {
        rb.words[word] = bits;
        if (bits)
            atomicOr((unsigned long long*)&rb.rowmask[row >> 6], 1ull << (row & 63));
    }
}

__global__ __launch_bounds__(kBlock) void label_write_kernel(const LabelWrite lw) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    label_write_clear(lw, v, (int64_t)gridDim.x * kBlock);
    if (v < lw.V)
        label_write_sample(lw, v);
}

LabelWrite label_write_args(fvv_ctx* ctx, const fvv_grid& g, uint8_t* occ, int32_t* labels) {
    LabelWrite lw;
    lw.sample_label = ctx->d_sample_label;
    lw.occ = occ;
    lw.labels = labels;
    lw.V = (int64_t)g.dims[0] * g.dims[1] * g.dims[2];
    lw.carve_blocks = 0u;
    const int64_t R = (int64_t)g.dims[1] * g.dims[2];
    lw.rb_words = ctx->d_rowbits;
    lw.rb_n = R * ((g.dims[0] + 63) / 64);
    lw.rowmask = ctx->d_rowmask;
    lw.rm_n = (R + 63) / 64;
    return lw;
}

RowBits row_bits(fvv_ctx* ctx, const fvv_grid& g) {
    return RowBits{ctx->d_rowbits, ctx->d_rowmask, (g.dims[0] + 63) / 64};
}

hipError_t launch_label(fvv_ctx* ctx, const fvv_grid& g, uint8_t* occ, int32_t* labels,
                        uint32_t t_np, uint32_t t_nb, fvv_roi* rois, uint32_t max_rois,
                        uint32_t* n_rois, bool seeded, const FrameJobs* frame, hipStream_t s) {
    LabelArgs a;
    a.rb = row_bits(ctx, g);
    a.nx = g.dims[0];
    a.ny = g.dims[1];
    a.nz = g.dims[2];
    a.g = RunArrays{ctx->d_rowmask, ctx->d_rmpre, ctx->d_rows, ctx->d_rs, ctx->d_x0,
                    ctx->d_x1,      nullptr,      ctx->d_rrow, ctx->d_runP};
    a.gstats = ctx->d_stats;
    a.sample_label = ctx->d_sample_label;
    a.t_np = t_np;
    a.t_nb = t_nb;
    a.rois = rois;
    a.max_rois = max_rois;
    a.n_rois = n_rois;
    a.status = ctx->d_status;
    a.pre = ctx->d_prefix;
    a.counter = ctx->d_counter;
    a.dcams = ctx->d_cams;
    if (!seeded) {
        const int64_t n_words = (int64_t)a.ny * a.nz * a.rb.wr;
        const int64_t blocks = (n_words * kWave + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(label_bitmap_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, occ,
                           a.nx, n_words, a.rb);
    }
    if (frame)
        hipLaunchKernelGGL(label_runs_kernel<true>, dim3(1), dim3(kLabelThreads), 0, s, a, *frame);
    else
        hipLaunchKernelGGL(label_runs_kernel<false>, dim3(1), dim3(kLabelThreads), 0, s, a,
                           FrameJobs{});
    if (!labels)
        return hipGetLastError();
    return launch_label_write(ctx, g, occ, labels, s);
}

// Labels and filtered occupancy of every sample (after launch_label).
hipError_t launch_label_write(fvv_ctx* ctx, const fvv_grid& g, uint8_t* occ, int32_t* labels,
                              hipStream_t s) {
    const LabelWrite lw = label_write_args(ctx, g, occ, labels);
    const unsigned vblocks = (unsigned)((lw.V + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(label_write_kernel, dim3(vblocks), dim3(kBlock), 0, s, lw);
    return hipGetLastError();
}

}  // namespace fvv

#ifdef FVV_LABEL_PHASES
// Measurement builds only: the last labelling's phase stamps to host memory
// (out: at least 10 entries).
extern "C" int32_t fvv_label_phase_stamps(uint64_t* out, int32_t n) {
    if (!out || n < fvv::kLabelPhases)
        return FVV_EINVAL;
    const hipError_t e = hipMemcpyFromSymbol(out, HIP_SYMBOL(fvv::label_phase_stamps),
                                             sizeof(uint64_t) * fvv::kLabelPhases);
    return e == hipSuccess ? FVV_OK : FVV_EDEVICE;
}
#endif
