// C ABI of the gfx950 visual-hull library: argument checks, the context's
// start-up allocation, and the launch sequence of each call.
#include <math.h>

#include <cmath>
#include <string.h>

#include <mutex>
#include <new>

#include "fvv_internal.h"
#include "measure.h"

using namespace fvv;

// An instantiated HIP graph (opaque to callers).
struct fvv_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace {

constexpr int64_t kMaxSamples = 0x7fffffffLL;
constexpr int32_t kMaxIndex = 1 << 24;  // (float)g is exact below this
// Spacing bound of a frame: index * spacing stays below 2^53 (exact in double)
constexpr int64_t kMaxSpacingUm = (int64_t)1 << 28;

bool finite3(const float* v) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }

int64_t grid_samples(const fvv_grid& g) {
    return (int64_t)g.dims[0] * (int64_t)g.dims[1] * (int64_t)g.dims[2];
}

bool grid_ok(const fvv_grid* g, int32_t index_limit) {
    if (!g)
        return false;
    if (!finite3(g->origin) || !isfinite(g->h) || !(g->h > 0.0f))
        return false;
    for (int a = 0; a < 3; ++a) {
        if (g->dims[a] < 1)
            return false;
        const int64_t lo = g->lo[a], hi = (int64_t)g->lo[a] + g->dims[a];
        if (lo <= -index_limit || hi >= index_limit)
            return false;
    }
    return grid_samples(*g) <= kMaxSamples;
}

// Cameras within the limits max_cams, max_w, max_h: same image size, finite P.
bool cams_within(int32_t max_cams, int32_t max_w, int32_t max_h, int32_t n,
                 const fvv_camera* cams) {
    if (!cams || n < 1 || n > FVV_MAX_CAMS || n > max_cams)
        return false;
    const int32_t W = cams[0].width, H = cams[0].height;
    if (W < 1 || H < 1 || W > max_w || H > max_h)
        return false;
    for (int c = 0; c < n; ++c) {
        if (cams[c].width != W || cams[c].height != H)
            return false;
        for (int e = 0; e < 12; ++e)
            if (!isfinite(cams[c].P[e]))
                return false;
    }
    return true;
}

bool cams_ok(const fvv_ctx* ctx, int32_t n, const fvv_camera* cams) {
    return cams_within(ctx->lim.max_cams, ctx->lim.max_w, ctx->lim.max_h, n, cams);
}

CamSet make_camset(int32_t n, const fvv_camera* cams, const fvv_grid* box = nullptr) {
    CamSet cs;
    memset(&cs, 0, sizeof(cs));
    cs.n = n;
    cs.W = cams[0].width;
    cs.H = cams[0].height;
    cs.wpr = (cs.W + 31) / 32;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    if (box)
        grid_box(*box, lo, hi);
    for (int c = 0; c < FVV_MAX_CAMS; ++c)
        cs.pad[c] = INFINITY;
    for (int c = 0; c < n; ++c) {
        for (int e = 0; e < 12; ++e)
            cs.P[c][e] = cams[c].P[e];
        if (box)
            cs.pad[c] = rounding_pad(cams[c].P, cs.W, cs.H, lo, hi);
    }
    return cs;
}

bool tile_ok(const fvv_tile* t) {
    if (!t)
        return true;
    if (!((t->tx == 64 && t->ty == 4) || (t->tx == 32 && t->ty == 8) ||
          (t->tx == 16 && t->ty == 16)))
        return false;
    if (!(t->tz == 1 || t->tz == 2 || t->tz == 4 || t->tz == 8))
        return false;
    return t->persistent_blocks >= 0 && t->persistent_blocks <= (1 << 20);
}

TileShape tile_of(const fvv_tile* t) {
    if (!t)
        return TileShape{64, 4, 4};
    return TileShape{t->tx, t->ty, t->tz};
}

int persistent_blocks(const fvv_ctx* ctx, const fvv_tile* t) {
    if (t && t->persistent_blocks > 0)
        return t->persistent_blocks;
    return ctx->n_cus * 8;
}

fvv_status dev(hipError_t e) { return e == hipSuccess ? FVV_OK : FVV_EDEVICE; }

int64_t floor_div64(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0)))
        q -= 1;
    return q;
}

int64_t ceil_div64(int64_t a, int64_t b) { return -floor_div64(-a, b); }

template <typename T>
hipError_t alloc(T** p, int64_t count) {
    if (count < 1)
        count = 1;
    return hipMalloc((void**)p, (size_t)count * sizeof(T));
}

bool soft_args_ok(fvv_ctx* ctx, const fvv_grid* grid, int32_t n_cams, const fvv_soft_camera* cams,
                  int32_t width, int32_t height, const float* d_logits) {
    return ctx && cams && d_logits && n_cams >= 1 && n_cams <= ctx->lim.max_cams && width >= 1 &&
           height >= 1 && width <= ctx->lim.max_w && height <= ctx->lim.max_h &&
           grid_ok(grid, kMaxIndex);
}

// The passes of fvv_surface on one lattice with the given scratch: its job
// and fine bitmap, the crossing edges, the exit points.
hipError_t launch_surface_single(const SurfaceScratch& sc, const fvv_job& job,
                                 const uint8_t* d_occ_fine, const CamSet& cs,
                                 const uint32_t* d_sils, int32_t n_steps, uint32_t* d_keys,
                                 float* d_xyz, uint32_t max_points, uint32_t* d_n_points,
                                 hipStream_t stream) {
    hipError_t e = launch_surface_prepare_single(sc, job, d_occ_fine, stream);
    // the exit points' pixel windows come from the tiled silhouettes, when the
    // scratch holds them
    const bool tiled = sc.tiles && tiled_sil_words(cs.n, cs.W, cs.H) <= sc.tile_cap;
    if (e == hipSuccess && tiled)
        e = launch_tile_sils(cs.n, cs.W, cs.H, d_sils, sc.tiles, nullptr, stream);
    if (e == hipSuccess)
        e = launch_edges(sc, sc.job_single, sc.counts_single + 3, d_keys, d_xyz, max_points,
                         sc.point_off_single, d_n_points, true, false, stream);
    if (e == hipSuccess)
        e = launch_bisect(sc.n_cus, sc.job_single, 1, sc.counts_single + 3, sc.point_off_single,
                          cs, d_sils, tiled ? sc.tiles : nullptr, n_steps, d_keys, d_xyz,
                          max_points, stream);
    return e;
}

// Argument checks shared by fvv_surface and fvv_surface_noalloc (the limits
// of the cameras and of the lattice's fine bitmap are the caller's).
bool surface_args_ok(const fvv_grid* roi, const uint8_t* d_occ_fine, int32_t n_cams,
                     const fvv_camera* cams, const uint32_t* d_sils, int32_t n_steps,
                     const uint32_t* d_keys, const float* d_xyz, uint32_t max_points,
                     const uint32_t* d_n_points) {
    return d_occ_fine && d_sils && d_keys && d_xyz && d_n_points && max_points >= 1 &&
           n_steps >= 1 && n_steps <= FVV_MAX_STEPS && cams && n_cams >= 1 &&
           grid_ok(roi, 1 << (23 - n_steps)) && grid_samples(*roi) <= 1431655765LL;
}

// ------------------------------------------------------------------ allocation-free surface
// The scratch of fvv_surface_noalloc: one array per device, laid out as the
// SurfaceScratch fields in this order, each at a 256-byte boundary.  Host
// code never passes `scratch` itself to a kernel (in host code the name is a
// host-side stand-in); it uses the device address that hipGetSymbolAddress
// returns for the current device.
constexpr int64_t kNoAllocItems = FVV_NOALLOC_BITMAP_WORDS / kEdgeWords + 2;
constexpr size_t round256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t kNaJob = 0;
constexpr size_t kNaPre = kNaJob + round256(sizeof(fvv_job));
constexpr size_t kNaCounts = kNaPre + round256(2 * sizeof(JobPrefix));
constexpr size_t kNaPointOff = kNaCounts + round256(4 * sizeof(uint32_t));
constexpr size_t kNaStatus = kNaPointOff + round256(2 * sizeof(uint32_t));
constexpr size_t kNaItems = kNaStatus + round256(sizeof(uint32_t));
constexpr size_t kNaBits = kNaItems + round256((size_t)kNoAllocItems * sizeof(uint32_t));
constexpr size_t kNaTiles = kNaBits + (size_t)FVV_NOALLOC_BITMAP_WORDS * sizeof(uint64_t);
constexpr size_t kNaBytes = kNaTiles + (size_t)FVV_NOALLOC_TILE_WORDS * sizeof(uint64_t);

constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
unsigned char* g_noalloc_ptr[kNoAllocDevices];   // device address of `scratch` per device
int g_noalloc_cus[kNoAllocDevices];

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {

// Device address and CU count of the current device's scratch (looked up
// once per device, under a lock).
hipError_t noalloc_scratch(SurfaceScratch* out) {
    int d = 0;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess)
        return e;
    if (d < 0 || d >= kNoAllocDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[d]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return e != hipSuccess ? e : hipErrorInvalidSymbol;
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d);
        if (e != hipSuccess)
            return e;
        g_noalloc_cus[d] = cus;
        g_noalloc_ptr[d] = (unsigned char*)ptr;
    }
    unsigned char* p = g_noalloc_ptr[d];
    out->job_single = (fvv_job*)(p + kNaJob);
    out->pre = (JobPrefix*)(p + kNaPre);
    out->counts_single = (uint32_t*)(p + kNaCounts);
    out->point_off_single = (uint32_t*)(p + kNaPointOff);
    out->status = (uint32_t*)(p + kNaStatus);
    out->item_cnt = (uint32_t*)(p + kNaItems);
    out->finebits = (uint64_t*)(p + kNaBits);
    out->word_edges = nullptr;
    out->tiles = (uint64_t*)(p + kNaTiles);
    out->tile_cap = FVV_NOALLOC_TILE_WORDS;
    out->n_cus = g_noalloc_cus[d];
    return hipSuccess;
}

// Capture what `record` enqueues on a fresh stream into an instantiated graph.
template <typename F>
fvv_status capture_graph(fvv_graph** out, F record) {
    if (!out)
        return FVV_EINVAL;
    *out = nullptr;
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
        return FVV_EDEVICE;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        hipStreamDestroy(s);
        return FVV_EDEVICE;
    }
    const fvv_status st = record(s);
    const hipError_t e = hipStreamEndCapture(s, &g);
    hipStreamDestroy(s);
    if (st != FVV_OK) {
        if (g)
            hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess || !g)
        return FVV_EDEVICE;
    hipGraphExec_t ex;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        hipGraphDestroy(g);
        return FVV_EDEVICE;
    }
    fvv_graph* r = new (std::nothrow) fvv_graph;
    if (!r) {
        hipGraphExecDestroy(ex);
        hipGraphDestroy(g);
        return FVV_ENOMEM;
    }
    r->graph = g;
    r->exec = ex;
    *out = r;
    return FVV_OK;
}

}  // namespace

extern "C" {

const char* fvv_status_str(fvv_status s) {
    switch (s) {
    case FVV_OK: return "ok";
    case FVV_EINVAL: return "invalid argument";
    case FVV_ECAPACITY: return "output capacity exceeded";
    case FVV_EDEVICE: return "device error";
    case FVV_ENOMEM: return "out of device memory";
    }
    return "unknown status";
}

void fvv_destroy(fvv_ctx* ctx) {
    if (!ctx)
        return;
    hipDeviceSynchronize();
    void* ptrs[] = {ctx->d_status, ctx->d_counter, ctx->d_rowbits, ctx->d_rowmask, ctx->d_rmpre,
                    ctx->d_rows, ctx->d_rs, ctx->d_x0, ctx->d_x1, ctx->d_rrow, ctx->d_runP,
                    ctx->d_stats,
                    ctx->d_sample_label, ctx->d_prefix, ctx->d_job_pad, ctx->d_soft_acc, ctx->d_mesh_table,
                    ctx->d_job_single, ctx->d_cams, ctx->d_finebits, ctx->d_item_cnt,
                    ctx->d_word_edges, ctx->d_tri_first, ctx->d_point_off_single,
                    ctx->d_counts_single, ctx->d_tsils, ctx->d_sany, ctx->d_rho};
    for (void* p : ptrs)
        if (p)
            hipFree(p);
    if (ctx->ev_join)
        hipEventDestroy(ctx->ev_join);
    if (ctx->ev_fine)
        hipEventDestroy(ctx->ev_fine);
    if (ctx->ev_edges)
        hipEventDestroy(ctx->ev_edges);
    if (ctx->side)
        hipStreamDestroy(ctx->side);
    delete ctx;
}

fvv_status fvv_create(fvv_ctx** out, const fvv_limits* lim) {
    if (!out)
        return FVV_EINVAL;
    *out = nullptr;
    if (!lim || lim->max_cams < 1 || lim->max_cams > FVV_MAX_CAMS || lim->max_w < 1 ||
        lim->max_h < 1 || lim->max_w > (1 << 16) || lim->max_h > (1 << 16) ||
        lim->max_coarse < 1 || lim->max_coarse > kMaxSamples || lim->max_fine < 1 ||
        lim->max_fine > ((int64_t)1 << 40) || lim->max_rois < 1 || lim->max_points < 1 ||
        lim->max_jobs < 1)
        return FVV_EINVAL;
    fvv_ctx* c = new (std::nothrow) fvv_ctx;
    if (!c)
        return FVV_ENOMEM;
    memset(c, 0, sizeof(*c));
    c->lim = *lim;
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipDeviceGetAttribute(&c->n_cus, hipDeviceAttributeMultiprocessorCount, c->device) !=
            hipSuccess) {
        delete c;
        return FVV_EDEVICE;
    }
    // a grid of at most V samples has at most V rows, V runs and V components,
    // and at most V + V/64 row-bitmap words (rows padded to whole words)
    const int64_t V = lim->max_coarse;
    const int64_t n_rowbits = V + V / 64 + 1, n_rowmask = V / 64 + 1;
    c->job_cap = (int64_t)(lim->max_jobs > lim->max_rois ? lim->max_jobs : lim->max_rois) + 2;
    // fine bitmaps: rows padded to whole words cost at most 1/4 + 1/64 word per
    // sample for lattices at least 4 samples wide (every frame ROI spans three
    // coarse cells); a single lattice of fvv_surface must fit as well
    c->bit_cap = lim->max_fine / 4 + lim->max_fine / 64 + (int64_t)lim->max_rois + 1;
    c->item_cap = c->bit_cap / kEdgeWords + (int64_t)lim->max_rois + 2;
    hipError_t e = hipSuccess;
#define A(ptr, n)                  \
    if (e == hipSuccess)           \
        e = alloc(&c->ptr, (n));
    A(d_status, 1)
    A(d_counter, kCounters)
    A(d_rowbits, n_rowbits)
    A(d_rowmask, n_rowmask)
    A(d_rmpre, n_rowmask)
    A(d_rows, V)
    A(d_rs, V + 1)
    A(d_x0, V)
    A(d_x1, V)
    A(d_rrow, V)
    A(d_runP, V)
    A(d_stats, (int64_t)(kStatsRow + 1) * V)
    A(d_sample_label, V)
    A(d_prefix, c->job_cap)
    A(d_job_pad, c->job_cap * FVV_MAX_CAMS)
    A(d_soft_acc, FVV_MAX_CAMS * 6)
    A(d_mesh_table, 1)
    A(d_job_single, 1)
    A(d_cams, FVV_MAX_CAMS)
    A(d_finebits, c->bit_cap)
    A(d_item_cnt, c->item_cap)
    A(d_word_edges, c->bit_cap)
    A(d_tri_first, c->item_cap)
    A(d_point_off_single, 2)
    A(d_counts_single, 4)
    A(d_tsils, tiled_sil_words(lim->max_cams, lim->max_w, lim->max_h))
    A(d_sany, sil_any_words(lim->max_cams, lim->max_w, lim->max_h))
    A(d_rho, c->job_cap * FVV_MAX_CAMS * kRhoPer)
#undef A
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&c->ev_fine, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&c->ev_edges, hipEventDisableTiming);
    if (e == hipSuccess) {
        MeshTable tbl;
        build_mesh_table(&tbl);
        e = hipMemcpy(c->d_mesh_table, &tbl, sizeof(tbl), hipMemcpyHostToDevice);
    }
    // scratch the kernels expect cleared (they clear it again after use)
    if (e == hipSuccess)
        e = hipMemset(c->d_status, 0, sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMemset(c->d_counter, 0, kCounters * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMemset(c->d_rowbits, 0, (size_t)n_rowbits * sizeof(uint64_t));
    if (e == hipSuccess)
        e = hipMemset(c->d_rowmask, 0, (size_t)n_rowmask * sizeof(uint64_t));
    if (e == hipSuccess)
        e = hipMemset(c->d_sany, 0,
                      (size_t)sil_any_words(lim->max_cams, lim->max_w, lim->max_h) *
                          sizeof(uint64_t));
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        fvv_destroy(c);
        return e == hipErrorOutOfMemory ? FVV_ENOMEM : FVV_EDEVICE;
    }
    *out = c;
    return FVV_OK;
}

fvv_status fvv_check(fvv_ctx* ctx, hipStream_t stream) {
    if (!ctx)
        return FVV_EINVAL;
    if (hipStreamSynchronize(stream) != hipSuccess)
        return FVV_EDEVICE;
    uint32_t flags = 0;
    if (hipMemcpy(&flags, ctx->d_status, sizeof(flags), hipMemcpyDeviceToHost) != hipSuccess)
        return FVV_EDEVICE;
    if (flags) {
        if (hipMemset(ctx->d_status, 0, sizeof(uint32_t)) != hipSuccess)
            return FVV_EDEVICE;
        if (hipDeviceSynchronize() != hipSuccess)
            return FVV_EDEVICE;
    }
    if (flags & kFlagJob)
        return FVV_EINVAL;
    return (flags & kFlagCapacity) ? FVV_ECAPACITY : FVV_OK;
}

fvv_status fvv_pack_silhouettes(fvv_ctx* ctx, int32_t n, int32_t width, int32_t height,
                                const uint8_t* d_masks, uint32_t* d_sils, hipStream_t stream) {
    if (!ctx || !d_masks || !d_sils || n < 1 || width < 1 || height < 1 ||
        width > ctx->lim.max_w || height > ctx->lim.max_h)
        return FVV_EINVAL;
    return dev(launch_pack(n, width, height, d_masks, d_sils, stream));
}

fvv_status fvv_carve(fvv_ctx* ctx, int32_t n_cams, const fvv_camera* cams, const uint32_t* d_sils,
                     const fvv_grid* grid, const fvv_tile* tile, uint8_t* d_occ,
                     hipStream_t stream) {
    if (!ctx || !d_sils || !d_occ || !cams_ok(ctx, n_cams, cams) || !grid_ok(grid, kMaxIndex) ||
        !tile_ok(tile))
        return FVV_EINVAL;
    const CamSet cs = make_camset(n_cams, cams, grid);   // pads over the lattice's box
    return dev(launch_carve(cs, d_sils, *grid, tile_of(tile), d_occ, nullptr, stream));
}

fvv_status fvv_label(fvv_ctx* ctx, const fvv_grid* grid, uint8_t* d_occ, int32_t* d_labels,
                     uint32_t t_np, uint32_t t_nb, fvv_roi* d_rois, uint32_t max_rois,
                     uint32_t* d_n_rois, hipStream_t stream) {
    if (!ctx || !grid || !d_occ || !d_labels || !d_rois || !d_n_rois || max_rois < 1 ||
        t_np > t_nb)
        return FVV_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (grid->dims[a] < 1)
            return FVV_EINVAL;
    if (grid_samples(*grid) > ctx->lim.max_coarse)
        return FVV_EINVAL;
    return dev(launch_label(ctx, *grid, d_occ, d_labels, t_np, t_nb, d_rois, max_rois, d_n_rois,
                            false, nullptr, stream));
}

fvv_status fvv_roi_grids(const fvv_grid* coarse, int64_t hc_um, int64_t hf_um,
                         const fvv_roi* rois, uint32_t n, fvv_grid* out) {
    if (!coarse || (n > 0 && (!rois || !out)) || hc_um < 1 || hf_um < 1)
        return FVV_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (coarse->dims[a] < 1)
            return FVV_EINVAL;
    const float h = (float)((double)hf_um * 1e-6);
    for (uint32_t t = 0; t < n; ++t) {
        fvv_grid g;
        for (int a = 0; a < 3; ++a) {
            if (rois[t].lo[a] < 0 || rois[t].hi[a] < rois[t].lo[a] ||
                rois[t].hi[a] >= coarse->dims[a])
                return FVV_EINVAL;
            const int64_t A = (int64_t)coarse->lo[a] + rois[t].lo[a] - 1;
            const int64_t B = (int64_t)coarse->lo[a] + rois[t].hi[a] + 1;
            int64_t f0 = floor_div64(A * hc_um, hf_um);
            int64_t f1 = ceil_div64(B * hc_um, hf_um);
            const int64_t fmin = ceil_div64((int64_t)coarse->lo[a] * hc_um, hf_um);
            const int64_t fmax =
                floor_div64(((int64_t)coarse->lo[a] + coarse->dims[a] - 1) * hc_um, hf_um);
            if (f0 < fmin)
                f0 = fmin;
            if (f1 > fmax)
                f1 = fmax;
            g.origin[a] = coarse->origin[a];
            g.lo[a] = (int32_t)f0;
            g.dims[a] = (int32_t)(f1 - f0 + 1);
        }
        g.h = h;
        out[t] = g;
    }
    return FVV_OK;
}

fvv_status fvv_surface(fvv_ctx* ctx, const fvv_grid* roi, const uint8_t* d_occ_fine,
                       int32_t n_cams, const fvv_camera* cams, const uint32_t* d_sils,
                       int32_t n_steps, uint32_t* d_keys, float* d_xyz, uint32_t max_points,
                       uint32_t* d_n_points, hipStream_t stream) {
    if (!ctx || !surface_args_ok(roi, d_occ_fine, n_cams, cams, d_sils, n_steps, d_keys, d_xyz,
                                 max_points, d_n_points) ||
        !cams_ok(ctx, n_cams, cams))
        return FVV_EINVAL;
    if (grid_samples(*roi) > ctx->lim.max_fine || fine_bitmap_words(*roi) > ctx->bit_cap)
        return FVV_EINVAL;
    const CamSet cs = make_camset(n_cams, cams, roi);
    fvv_job job;
    memset(&job, 0, sizeof(job));
    job.grid = *roi;
    job.n_cams = n_cams;
    job.width = cs.W;
    job.height = cs.H;
    return dev(launch_surface_single(surface_scratch(ctx), job, d_occ_fine, cs, d_sils, n_steps,
                                     d_keys, d_xyz, max_points, d_n_points, stream));
}

fvv_status fvv_surface_noalloc(const fvv_grid* roi, const uint8_t* d_occ_fine, int32_t n_cams,
                               const fvv_camera* cams, const uint32_t* d_sils, int32_t n_steps,
                               uint32_t* d_keys, float* d_xyz, uint32_t max_points,
                               uint32_t* d_n_points, hipStream_t stream) {
    if (!surface_args_ok(roi, d_occ_fine, n_cams, cams, d_sils, n_steps, d_keys, d_xyz,
                         max_points, d_n_points) ||
        !cams_within(FVV_MAX_CAMS, 1 << 16, 1 << 16, n_cams, cams) ||
        fine_bitmap_words(*roi) > FVV_NOALLOC_BITMAP_WORDS)
        return FVV_EINVAL;
    SurfaceScratch sc;
    if (noalloc_scratch(&sc) != hipSuccess)
        return FVV_EDEVICE;
    const CamSet cs = make_camset(n_cams, cams, roi);
    fvv_job job;
    memset(&job, 0, sizeof(job));
    job.grid = *roi;
    job.n_cams = n_cams;
    job.width = cs.W;
    job.height = cs.H;
    return dev(launch_surface_single(sc, job, d_occ_fine, cs, d_sils, n_steps, d_keys, d_xyz,
                                     max_points, d_n_points, stream));
}

fvv_status fvv_carve_batched(fvv_ctx* ctx, const fvv_job* d_jobs, uint32_t n_jobs,
                             const fvv_camera* d_cams, const uint32_t* d_sils,
                             uint8_t* d_occ_out, const fvv_tile* tile, hipStream_t stream) {
    if (!ctx || !d_jobs || !d_cams || !d_sils || !d_occ_out || n_jobs < 1 ||
        n_jobs > ctx->lim.max_jobs || !tile_ok(tile))
        return FVV_EINVAL;
    return dev(launch_carve_batched(ctx, d_jobs, n_jobs, d_cams, d_sils, d_occ_out, nullptr,
                                    tile_of(tile), persistent_blocks(ctx, tile), false, stream));
}

fvv_status fvv_mesh(fvv_ctx* ctx, const fvv_grid* grid, const uint8_t* d_occ,
                    const uint32_t* d_keys, const uint32_t* d_n_keys, uint32_t max_keys,
                    uint32_t* d_tris, uint32_t max_tris, uint32_t* d_n_tris, hipStream_t stream) {
    if (!ctx || !grid || !d_occ || !d_keys || !d_n_keys || !d_tris || !d_n_tris || max_keys < 1 ||
        max_tris < 1)
        return FVV_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (grid->dims[a] < 1)
            return FVV_EINVAL;
    // keys 3*lin+axis stay 32-bit; the lattice's fine bitmap fits the scratch
    if (grid_samples(*grid) > (int64_t)0x55555555 || fine_bitmap_words(*grid) > ctx->bit_cap)
        return FVV_EINVAL;
    return dev(launch_mesh(ctx, *grid, d_occ, d_keys, d_n_keys, max_keys, d_tris, max_tris,
                           d_n_tris, stream));
}

fvv_status fvv_isovalue(fvv_ctx* ctx, const fvv_grid* grid, const uint8_t* d_occ, int32_t n_cams,
                        const fvv_camera* cams, const uint32_t* d_sils, const uint32_t* d_keys,
                        const uint32_t* d_n_keys, uint32_t max_keys, float* d_lambda,
                        float* d_xyz, hipStream_t stream) {
    if (!ctx || !d_occ || !d_sils || !d_keys || !d_n_keys || !d_lambda || max_keys < 1 ||
        !cams_ok(ctx, n_cams, cams) || !grid_ok(grid, kMaxIndex))
        return FVV_EINVAL;
    if (grid_samples(*grid) > (int64_t)0x55555555)
        return FVV_EINVAL;
    const CamSet cs = make_camset(n_cams, cams);
    return dev(launch_isovalue(ctx, *grid, d_occ, cs, d_sils, d_keys, d_n_keys, max_keys, d_lambda,
                               d_xyz, stream));
}

fvv_status fvv_visibility(fvv_ctx* ctx, int32_t n_cams, const fvv_camera* cams,
                          const float* d_xyz, const uint32_t* d_n_vertices, uint32_t max_vertices,
                          const uint32_t* d_tris, const uint32_t* d_n_tris, uint32_t max_tris,
                          float t_v, float* d_depth, uint32_t* d_vis, hipStream_t stream) {
    if (!ctx || !d_xyz || !d_n_vertices || !d_tris || !d_n_tris || !d_depth || !d_vis ||
        max_vertices < 1 || max_tris < 1 || !isfinite(t_v) || !cams_ok(ctx, n_cams, cams))
        return FVV_EINVAL;
    const CamSet cs = make_camset(n_cams, cams);
    return dev(launch_visibility(ctx, cs, d_xyz, d_n_vertices, max_vertices, d_tris, d_n_tris,
                                 max_tris, t_v, d_depth, d_vis, stream));
}

fvv_status fvv_gather_peak(fvv_ctx* ctx, const uint32_t* d_table, uint32_t n_words,
                           uint32_t* d_sink, int32_t reps, double* words_per_s,
                           hipStream_t stream) {
    if (!ctx || !d_table || !d_sink || !words_per_s || n_words < 64 || reps < 1 || reps > 1000)
        return FVV_EINVAL;
    const uint32_t blocks = (uint32_t)(ctx->n_cus * 64 < 16384 ? ctx->n_cus * 64 : 16384);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return FVV_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return FVV_EDEVICE;
    }
    fvv_status st = dev(launch_gather_peak(ctx, d_table, n_words, d_sink, blocks, stream));
    if (st == FVV_OK)
        st = dev(hipEventRecord(e0, stream));
    for (int32_t r = 0; r < reps && st == FVV_OK; ++r)
        st = dev(launch_gather_peak(ctx, d_table, n_words, d_sink, blocks, stream));
    if (st == FVV_OK)
        st = dev(hipEventRecord(e1, stream));
    if (st == FVV_OK)
        st = dev(hipEventSynchronize(e1));
    float ms = 0.0f;
    if (st == FVV_OK)
        st = dev(hipEventElapsedTime(&ms, e0, e1));
    if (st == FVV_OK)
        *words_per_s = (double)gather_peak_words(blocks) * reps / ((double)ms * 1e-3);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return st;
}

// ------------------------------------------------------------------ soft hull
fvv_status fvv_soft_forward(fvv_ctx* ctx, const fvv_grid* grid, int32_t n_cams,
                            const fvv_soft_camera* cams, int32_t width, int32_t height,
                            const float* d_logits, const float* d_target, float* d_occ,
                            double* d_loss, hipStream_t stream) {
    if (!soft_args_ok(ctx, grid, n_cams, cams, width, height, d_logits) || (!d_occ && !d_loss) ||
        (d_loss && !d_target))
        return FVV_EINVAL;
    SoftCamSet cs;
    SoftJacobians jac;
    if (!make_soft_cams(n_cams, width, height, cams, &cs, &jac))
        return FVV_EINVAL;
    return dev(launch_soft_forward(ctx, cs, *grid, d_logits, d_target, d_occ, d_loss, stream));
}

fvv_status fvv_soft_backward(fvv_ctx* ctx, const fvv_grid* grid, int32_t n_cams,
                             const fvv_soft_camera* cams, int32_t width, int32_t height,
                             const float* d_logits, const float* d_target,
                             const float* d_grad_occ, const double* d_scale,
                             float* d_grad_logits, double* d_grad_pose, hipStream_t stream) {
    if (!soft_args_ok(ctx, grid, n_cams, cams, width, height, d_logits) || !d_grad_logits ||
        !d_grad_pose || (!d_target) == (!d_grad_occ))
        return FVV_EINVAL;
    SoftCamSet cs;
    SoftJacobians jac;
    if (!make_soft_cams(n_cams, width, height, cams, &cs, &jac))
        return FVV_EINVAL;
    return dev(launch_soft_backward(ctx, cs, jac, *grid, d_logits, d_target, d_grad_occ, d_scale,
                                    d_grad_logits, d_grad_pose, stream));
}

fvv_status fvv_frame(fvv_ctx* ctx, const fvv_frame_params* p, const uint8_t* d_masks,
                     uint32_t* d_sils, const fvv_frame_out* o, hipEvent_t* events,
                     hipStream_t stream) {
    if (!ctx || !p || !o || !d_sils || !cams_ok(ctx, p->n_cams, p->cams) ||
        !grid_ok(&p->coarse, kMaxIndex) || p->hc_um < 1 || p->hf_um < 1 ||
        p->hc_um > kMaxSpacingUm || p->hf_um > kMaxSpacingUm || p->t_np > p->t_nb ||
        p->n_steps < 1 || p->n_steps > FVV_MAX_STEPS || !tile_ok(&p->coarse_tile) ||
        !tile_ok(&p->fine_tile) ||
        (p->exit_estimator != FVV_EXIT_BISECTION && p->exit_estimator != FVV_EXIT_BRESENHAM))
        return FVV_EINVAL;
    if (!o->d_occ_coarse || !o->d_labels || !o->d_rois || !o->d_jobs || !o->d_occ_fine ||
        !o->d_keys || !o->d_xyz || !o->d_point_off || !o->d_counts || o->max_rois < 1 ||
        o->max_rois > ctx->lim.max_rois || o->max_fine < 1 || o->max_fine > ctx->lim.max_fine ||
        o->max_points < 1)
        return FVV_EINVAL;
    const bool mesh = o->d_tris != nullptr;
    if (mesh && (!o->d_tri_off || o->max_tris < 1))
        return FVV_EINVAL;
    if (grid_samples(p->coarse) > ctx->lim.max_coarse)
        return FVV_EINVAL;
    // every fine index must stay exact through the bisection
    for (int a = 0; a < 3; ++a) {
        const int64_t hi = ((int64_t)p->coarse.lo[a] + p->coarse.dims[a]) * p->hc_um / p->hf_um + 2;
        const int64_t lo = (int64_t)p->coarse.lo[a] * p->hc_um / p->hf_um - 2;
        const int64_t lim = (int64_t)1 << (23 - p->n_steps);
        if (hi >= lim || lo <= -lim)
            return FVV_EINVAL;
    }
    if (events)
        for (int i = 0; i < FVV_FRAME_EVENTS; ++i)
            if (!events[i])
                return FVV_EINVAL;
    // every fine sample of the frame lies in the coarse lattice's box (widened
    // by one cell against the rounding of the fine coordinates)
    fvv_grid wide = p->coarse;
    for (int a = 0; a < 3; ++a) {
        wide.lo[a] -= 1;
        wide.dims[a] += 2;
    }
    const CamSet cs = make_camset(p->n_cams, p->cams, &wide);
    const float h_fine = (float)((double)p->hf_um * 1e-6);
    const TileShape ct = tile_of(&p->coarse_tile), ft = tile_of(&p->fine_tile);
    // the fine carve's workgroups: the tile's count, else 16 per CU (a frame's
    // ~3e3 tiles as single-tile workgroups; measured faster than 8 or 24 per CU)
    const int blocks = p->fine_tile.persistent_blocks > 0 ? p->fine_tile.persistent_blocks
                                                          : ctx->n_cus * 16;
    auto mark = [&](int i) {
        if (events)
            (void)hipEventRecord(events[i], stream);
    };
    // the kernels' own start and end times: fine carve, exit points
    auto kev = [&](int i) -> hipEvent_t { return events ? events[FVV_FRAME_STAGE_EVENTS + i] : nullptr; };
    hipError_t e = hipSuccess;
    mark(0);
    // a large coarse lattice is carved in two passes, the first rejecting
    // whole boxes by the silhouettes' non-empty blocks (the list of the kept
    // ones in the labelling's sample-label scratch, unused until the
    // labelling, which clears their count)
    const bool two_pass = ct.tz != 4 && (uint64_t)grid_samples(p->coarse) >= kRejectMinSamples;
    const CarveReject rej{SilAny{ctx->d_sany, sil_any_bw(cs.W), (cs.H + 7) / 8},
                          reinterpret_cast<uint32_t*>(ctx->d_sample_label),
                          ctx->d_counter + kCounterBoxes, ctx->n_cus};
    // the packed rows, the 8 x 8-pixel blocks the fine carve and the exit
    // points read, and (two passes) which of the blocks are non-empty
    uint64_t* const sany = two_pass ? ctx->d_sany : nullptr;
    if (d_masks)
        e = launch_pack_tiled(p->n_cams, cs.W, cs.H, d_masks, d_sils, ctx->d_tsils, sany, stream);
    else
        e = launch_tile_sils(p->n_cams, cs.W, cs.H, d_sils, ctx->d_tsils, sany, stream);
    mark(1);
    // the coarse carve also fills the labelling's row bitmap
    const RowBits rb = row_bits(ctx, p->coarse);
    if (e == hipSuccess)
        e = launch_carve(cs, d_sils, p->coarse, ct, o->d_occ_coarse, &rb, stream,
                         two_pass ? &rej : nullptr);
    mark(2);
    // labelling; its selection kernel also lays out the fine jobs of the ROIs
    FrameJobs fj;
    fj.cams = cs;
    fj.coarse = p->coarse;
    fj.hc_um = p->hc_um;
    fj.hf_um = p->hf_um;
    fj.h_fine = h_fine;
    fj.jobs = o->d_jobs;
    fj.max_fine = o->max_fine;
    fj.counts = o->d_counts;
    fj.tile_x = ft.tx;
    fj.tile_z = ft.tz;
    fj.blocks = (uint32_t)blocks;
    fj.bit_cap = ctx->bit_cap;
    fj.rho = ctx->d_rho;
    if (e == hipSuccess)
        e = launch_label(ctx, p->coarse, o->d_occ_coarse, nullptr, p->t_np, p->t_nb, o->d_rois,
                         o->max_rois, o->d_counts + 0, true, &fj, stream);
    mark(3);
    // the fine carve; the grid pass writing labels and the filtered coarse
    // occupancy rides in its launch (a branch to the side stream and back, or
    // a launch of its own, costs more than the pass)
    if (e == hipSuccess)
        e = launch_carve_frame(ctx, o->d_jobs, (int)o->max_rois, cs, d_sils, ctx->d_tsils,
                               o->d_occ_fine, ctx->d_finebits, ft, blocks, p->coarse,
                               o->d_occ_coarse, o->d_labels, stream, kev(0), kev(1));
    mark(4);
    // the mesh also runs on the side branch: its count once the fine bitmaps
    // are there, its triangles once the crossing edges are, beside the exit
    // points
    const uint32_t* n_jobs = o->d_counts + 3;
    if (mesh && e == hipSuccess)
        e = hipEventRecord(ctx->ev_fine, stream);
    if (mesh && e == hipSuccess)
        e = hipStreamWaitEvent(ctx->side, ctx->ev_fine, 0);
    if (mesh && e == hipSuccess)
        e = launch_mesh_count(ctx, o->d_jobs, n_jobs, 0, ctx->side);
    if (e == hipSuccess)
        e = launch_edges(surface_scratch(ctx), o->d_jobs, n_jobs, o->d_keys, o->d_xyz, o->max_points,
                         o->d_point_off, o->d_counts + 2, true, mesh, stream);
    mark(5);
    if (mesh && e == hipSuccess)
        e = hipEventRecord(ctx->ev_edges, stream);
    if (mesh && e == hipSuccess)
        e = hipStreamWaitEvent(ctx->side, ctx->ev_edges, 0);
    if (mesh && e == hipSuccess)
        e = launch_mesh_write(ctx, o->d_jobs, n_jobs, o->d_keys, o->d_counts + 2, o->max_points,
                              false, o->d_tris, o->max_tris, o->d_tri_off, nullptr, 0,
                              ctx->side);
    if (mesh && e == hipSuccess)
        e = hipEventRecord(ctx->ev_join, ctx->side);
    if (e == hipSuccess && p->exit_estimator == FVV_EXIT_BRESENHAM)
        e = launch_isovalue_jobs(ctx, o->d_jobs, n_jobs, o->d_point_off, cs, d_sils, o->d_keys,
                                 o->d_xyz, o->max_points, stream, kev(2), kev(3));
    else if (e == hipSuccess)
        e = launch_bisect(ctx->n_cus, o->d_jobs, (int)o->max_rois, n_jobs, o->d_point_off, cs,
                          d_sils, ctx->d_tsils, p->n_steps, o->d_keys, o->d_xyz, o->max_points,
                          stream, kev(2), kev(3));
    if (mesh && e == hipSuccess)
        e = hipStreamWaitEvent(stream, ctx->ev_join, 0);
    mark(6);
    return dev(e);
}

fvv_status fvv_frame_graph_create(fvv_ctx* ctx, const fvv_frame_params* p,
                                  const uint8_t* d_masks, uint32_t* d_sils,
                                  const fvv_frame_out* o, fvv_graph** out) {
    return capture_graph(out, [&](hipStream_t s) {
        return fvv_frame(ctx, p, d_masks, d_sils, o, nullptr, s);
    });
}

fvv_status fvv_carve_batched_graph_create(fvv_ctx* ctx, const fvv_job* d_jobs, uint32_t n_jobs,
                                          const fvv_camera* d_cams, const uint32_t* d_sils,
                                          uint8_t* d_occ_out, const fvv_tile* tile,
                                          fvv_graph** out) {
    return capture_graph(out, [&](hipStream_t s) {
        return fvv_carve_batched(ctx, d_jobs, n_jobs, d_cams, d_sils, d_occ_out, tile, s);
    });
}

fvv_status fvv_tune_carve_batched(fvv_ctx* ctx, const fvv_job* d_jobs, uint32_t n_jobs,
                                  const fvv_camera* d_cams, const uint32_t* d_sils,
                                  uint8_t* d_occ_out, const fvv_tile* cands, uint32_t n_cands,
                                  int32_t reps, float* ms, uint32_t* best, hipStream_t stream) {
    if (!ctx || !cands || n_cands < 1 || reps < 1 || reps > 1000 || !ms || !best)
        return FVV_EINVAL;
    for (uint32_t i = 0; i < n_cands; ++i)
        if (!tile_ok(&cands[i]))
            return FVV_EINVAL;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return FVV_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return FVV_EDEVICE;
    }
    fvv_status st = FVV_OK;
    uint32_t arg = 0;
    for (uint32_t i = 0; i < n_cands && st == FVV_OK; ++i) {
        // one untimed call, then reps calls between the events
        st = fvv_carve_batched(ctx, d_jobs, n_jobs, d_cams, d_sils, d_occ_out, &cands[i], stream);
        if (st == FVV_OK)
            st = dev(hipEventRecord(e0, stream));
        for (int32_t r = 0; r < reps && st == FVV_OK; ++r)
            st = fvv_carve_batched(ctx, d_jobs, n_jobs, d_cams, d_sils, d_occ_out, &cands[i],
                                   stream);
        if (st == FVV_OK)
            st = dev(hipEventRecord(e1, stream));
        if (st == FVV_OK)
            st = dev(hipEventSynchronize(e1));
        float t = 0.0f;
        if (st == FVV_OK)
            st = dev(hipEventElapsedTime(&t, e0, e1));
        if (st == FVV_OK) {
            ms[i] = t / (float)reps;
            if (ms[i] < ms[arg])
                arg = i;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st == FVV_OK)
        *best = arg;
    return st;
}

fvv_status fvv_graph_launch(fvv_graph* g, hipStream_t stream) {
    if (!g)
        return FVV_EINVAL;
    return dev(hipGraphLaunch(g->exec, stream));
}

void fvv_graph_destroy(fvv_graph* g) {
    if (!g)
        return;
    hipGraphExecDestroy(g->exec);
    hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"
