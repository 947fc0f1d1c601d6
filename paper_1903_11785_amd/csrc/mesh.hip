// Marching-cubes triangles of one lattice on gfx950 (Sec. II-C: with a vertex
// on every crossing edge, the isosurface follows the marching-cubes
// configurations and is expressed as triangles).  The configurations are
// those of the face rule stated in include/fvv.h (fvv_mesh), tabulated once
// per context for the 256 corner patterns.
//
// Table construction: every cell face is walked around its corners counter-
// clockwise as seen from outside the cell.  A face edge leading from an
// occupied corner to an empty one is an exit, the reverse an entry; the
// segment of an exit starts at the nearest entry before it in that walk.
// This links an entry to the exit that cuts off the occupied corners between
// them (with two diagonal occupied corners, each is cut off alone) and puts
// the face's occupied part on the segment's right seen from outside.  The
// linked edges form loops, each fanned from the first vertex, in loop order
// from its smallest cell edge, none of whose two faces the loop crosses twice.
#include <string.h>

#include "fvv_internal.h"

namespace fvv {

// Corner cycles of the six faces, counter-clockwise seen from outside
// (corner b = dx + 2 dy + 4 dz): x = 0, x = 1, y = 0, y = 1, z = 0, z = 1.
static const int kFaceCycle[6][4] = {{0, 4, 6, 2}, {1, 3, 7, 5}, {0, 1, 5, 4},
                                     {2, 6, 7, 3}, {0, 2, 3, 1}, {4, 5, 7, 6}};

// Cell edge joining corners b0 and b1 (one coordinate apart): 4 a + u + 2 v.
static int cell_edge_of(int b0, int b1) {
    const int diff = b0 ^ b1;
    const int a = diff == 1 ? 0 : (diff == 2 ? 1 : 2);
    const int lo = b0 & b1;                     // the corner with coordinate a = 0
    int uv[2], m = 0;
    for (int d = 0; d < 3; ++d)
        if (d != a)
            uv[m++] = (lo >> d) & 1;
    return 4 * a + uv[0] + 2 * uv[1];
}

void build_mesh_table(MeshTable* t) {
    memset(t, 0, sizeof(*t));
    for (int cs = 0; cs < 256; ++cs) {
        int next[12], entry_face[12], exit_face[12];
        for (int e = 0; e < 12; ++e)
            next[e] = entry_face[e] = exit_face[e] = -1;
        for (int f = 0; f < 6; ++f) {
            int edge[4], kind[4];   // kind: +1 exit, -1 entry, 0 none
            for (int i = 0; i < 4; ++i) {
                const int q0 = kFaceCycle[f][i], q1 = kFaceCycle[f][(i + 1) & 3];
                const int in0 = (cs >> q0) & 1, in1 = (cs >> q1) & 1;
                edge[i] = cell_edge_of(q0, q1);
                kind[i] = in0 && !in1 ? 1 : (!in0 && in1 ? -1 : 0);
            }
            for (int i = 0; i < 4; ++i) {
                if (kind[i] != 1)
                    continue;
                for (int back = 1; back < 4; ++back) {
                    const int j = (i - back + 4) & 3;
                    if (kind[j] == -1) {
                        next[edge[j]] = edge[i];
                        entry_face[edge[j]] = f;
                        exit_face[edge[i]] = f;
                        break;
                    }
                }
            }
        }
        bool seen[12] = {false};
        int ntri = 0;
        for (int e0 = 0; e0 < 12; ++e0) {
            if (next[e0] < 0 || seen[e0])
                continue;
            int loop[12], m = 0;
            for (int x = e0; !seen[x]; x = next[x]) {
                seen[x] = true;
                loop[m++] = x;
            }
            int per_face[6] = {0, 0, 0, 0, 0, 0};
            for (int q = 0; q < m; ++q)
                ++per_face[entry_face[loop[q]]];   // the segment leaving loop[q]
            int apex = 0;
            for (int q = 0; q < m; ++q)
                if (per_face[entry_face[loop[q]]] < 2 && per_face[exit_face[loop[q]]] < 2) {
                    apex = q;
                    break;
                }
            for (int q = 1; q + 1 < m; ++q) {
                t->edge[cs][3 * ntri + 0] = (uint8_t)loop[apex];
                t->edge[cs][3 * ntri + 1] = (uint8_t)loop[(apex + q) % m];
                t->edge[cs][3 * ntri + 2] = (uint8_t)loop[(apex + q + 1) % m];
                ++ntri;
            }
        }
        t->count[cs] = (uint8_t)ntri;
    }
}

// ------------------------------------------------------------------ kernels
// The passes run over the fine bitmaps of the jobs with the work items of the
// crossing-edge compaction (kEdgeWords words of one lattice, one word per
// thread).  A word's cells are those whose first corner is one of its
// samples: bit b is the cell (64 q + b, y, z), with corners in the rows
// (y + dy, z + dz), m = dy + 2 dz, at bits b and b + 1 (bit 0 of the next word
// for b = 63).  Cells in linear order are words in order, then bits in order,
// so triangles come out by cell in linear order.

// The four rows of a word's cells: samples x (r) and x + 1 (s) of each, and
// the cells that have both occupied and empty corners.
struct CellRows {
    uint64_t r[4], s[4];
    uint64_t mixed;
};

__device__ __forceinline__ CellRows cell_rows(const uint64_t* __restrict__ bits, int64_t w,
                                              const int32_t* d, int32_t wr) {
    CellRows c;
    const int64_t row = w / wr;
    const int32_t q = (int32_t)(w - row * wr);
    const bool last = q == wr - 1;
    const int32_t y = (int32_t)(row % d[1]);
    const int32_t z = (int32_t)(row / d[1]);
    const bool cells = y + 1 < d[1] && z + 1 < d[2];
    const int64_t slab = (int64_t)wr * d[1];
    // rows past the lattice are never read: their loads repeat this word
    const int64_t wm[4] = {w, cells ? w + wr : w, cells ? w + slab : w,
                           cells ? w + wr + slab : w};
    uint64_t any = 0, all = ~0ull;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        c.r[m] = bits[wm[m]];
        const uint64_t nx = last ? 0ull : bits[wm[m] + 1];
        c.s[m] = (c.r[m] >> 1) | (nx << 63);
        any |= c.r[m] | c.s[m];
        all &= c.r[m] & c.s[m];
    }
    // cell x needs sample x + 1 in the lattice: in the last word bits
    // [0, nx - 64 q - 1) are cells (at most 63)
    const int32_t in_last = d[0] - 64 * q - 1;
    const uint64_t cellmask = last ? ((1ull << in_last) - 1ull) : ~0ull;
    c.mixed = cells ? (any & ~all) & cellmask : 0ull;
    return c;
}

// Corner pattern of the cell at bit b (corner dx + 2 dy + 4 dz = dx + 2 m).
__device__ __forceinline__ int cell_pattern(const CellRows& c, int b) {
    int cs = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m)
        cs |= (int)((c.r[m] >> b) & 1u) << (2 * m) | (int)((c.s[m] >> b) & 1u) << (2 * m + 1);
    return cs;
}

__device__ __forceinline__ void load_table(const MeshTable* __restrict__ tbl, MeshTable* s_tbl) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(tbl);
    uint32_t* dst = reinterpret_cast<uint32_t*>(s_tbl);
    for (int i = threadIdx.x; i < (int)(sizeof(MeshTable) / 4); i += kBlock)
        dst[i] = src[i];
    __syncthreads();
}

__device__ __forceinline__ uint32_t cell_triangles(const CellRows& c, const MeshTable& t) {
    uint32_t n = 0;
    for (uint64_t b = c.mixed; b; b &= b - 1)
        n += t.count[cell_pattern(c, __ffsll((unsigned long long)b) - 1)];
    return n;
}

// Per work item: its number of triangles.  The last workgroup to finish
// (counted on `arrived`, zero on entry) turns the counts into each item's
// first triangle, an exclusive scan in place, and sets `arrived` back to zero.
__global__ __launch_bounds__(kBlock) void mesh_count_kernel(const fvv_job* __restrict__ jobs,
                                                            const JobPrefix* __restrict__ pre,
                                                            const uint32_t* __restrict__ n_jobs_p,
                                                            const uint64_t* __restrict__ bits,
                                                            const MeshTable* __restrict__ tbl,
                                                            uint64_t* __restrict__ tri_first,
                                                            uint32_t* __restrict__ arrived) {
    __shared__ uint32_t table[kJobTable];
    __shared__ uint32_t scratch[kBlock / kWave];
    __shared__ uint64_t scratch64[kBlock / kWave];
    __shared__ MeshTable s_tbl;
    __shared__ bool s_last;
    const int nj = (int)*n_jobs_p;
    const uint32_t items_all = pre[nj].item_off;
    if (blockIdx.x >= items_all)           // no item for this workgroup
        return;
    const uint32_t active = gridDim.x < items_all ? gridDim.x : items_all;
    load_table(tbl, &s_tbl);
    const ItemJobs ij = load_item_jobs(pre, nj, table);
    const uint32_t n_items = ij.first_item(nj);
    for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int jb = ij.job_of(item);
        const fvv_grid g = jobs[jb].grid;
        const int64_t w = (int64_t)(item - ij.first_item(jb)) * kEdgeWords + threadIdx.x;
        uint32_t n = 0;
        if (w < fine_bitmap_words(g))
            n = cell_triangles(cell_rows(bits + pre[jb].bit_off, w, g.dims, (g.dims[0] + 63) / 64),
                               s_tbl);
        uint32_t total;
        block_exclusive_sum<kBlock>(n, scratch, &total);
        if (threadIdx.x == 0)
            tri_first[item] = total;
    }
    __threadfence();                        // the counts, before the arrival
    __syncthreads();
    if (threadIdx.x == 0)
        s_last = atomicAdd(arrived, 1u) == active - 1;
    __syncthreads();
    if (!s_last)
        return;
    __threadfence();                        // every workgroup's counts, after its arrival
    uint64_t carry = 0;
    for (uint32_t b0 = 0; b0 < n_items; b0 += kBlock) {
        const uint32_t i = b0 + threadIdx.x;
        const uint64_t v = i < n_items
                               ? __hip_atomic_load(tri_first + i, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT)
                               : 0ull;
        uint64_t all;
        const uint64_t ex = block_exclusive_sum64<kBlock>(v, scratch64, &all);
        if (i < n_items)
            tri_first[i] = carry + ex;
        carry += all;
    }
    if (threadIdx.x == 0)
        *arrived = 0;
}

// A cell listed for the write pass: the lane of its word in the wave, its bit,
// its corner pattern and its first triangle (relative to the work item).
constexpr int kCellRecs = 256;   // per wave and pass

__device__ __forceinline__ uint2 cell_rec(int lane, int b, int cs, uint32_t t) {
    return make_uint2((uint32_t)lane | (uint32_t)b << 6 | (uint32_t)cs << 12, t);
}

// Per work item: its first triangle from the count pass, then a scan over the
// threads gives each word's first triangle.  The words' cells
// are then spread over the wave's lanes: each lane lists its word's cells
// (bit, pattern, first triangle) in the wave's LDS records, and every lane
// takes every 64th record.  A vertex on cell edge 4 a + u + 2 v has its edge's
// first sample at (dx, dy, dz) with d_a = 0 and (u, v) on the other two axes;
// the owning word's WordEdges give its position (each word's four owners in
// rows y..y+1, z..z+1 are staged in LDS; the next word's, needed at b = 63
// only, are read from memory).  The 12 positions of a cell
// go through LDS (one column per thread) so that the table's runtime edge
// numbers index them; a crossing edge whose position is past the keys (or,
// kVerify, holds another key) becomes 0xffffffff.
template <bool kVerify>
__global__ __launch_bounds__(kBlock) void mesh_write_kernel(
    const fvv_job* __restrict__ jobs, const JobPrefix* __restrict__ pre,
    const uint32_t* __restrict__ n_jobs_p, const uint64_t* __restrict__ bits,
    const MeshTable* __restrict__ tbl, const uint64_t* __restrict__ tri_first,
    const WordEdges* __restrict__ wedges, const uint32_t* __restrict__ keys,
    const uint32_t* __restrict__ n_keys_p, uint32_t max_keys, uint32_t* __restrict__ tris,
    uint32_t max_tris, uint32_t* __restrict__ tri_off, uint32_t* __restrict__ n_tris,
    uint32_t* __restrict__ status) {
    constexpr int kWaves = kBlock / kWave;
    __shared__ uint32_t table[kJobTable];
    __shared__ uint32_t scratch[kWaves];
    __shared__ MeshTable s_tbl;
    __shared__ uint32_t s_pos[12][kBlock];
    __shared__ uint2 s_rec[kWaves][kCellRecs];
    __shared__ WordEdges s_own[4][kBlock];   // each word's owners in rows m, this q
    const int nj = (int)*n_jobs_p;
    const uint32_t items_all = pre[nj].item_off;
    if (items_all == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
        if (tri_off)
            for (int j = 0; j <= nj; ++j)
                tri_off[j] = 0;
        if (n_tris)
            *n_tris = 0;
    }
    if (blockIdx.x >= items_all)           // no item for this workgroup
        return;
    load_table(tbl, &s_tbl);
    const ItemJobs ij = load_item_jobs(pre, nj, table);
    const uint32_t n_items = ij.first_item(nj);
    const uint32_t nk_all = *n_keys_p;
    const uint32_t nk = nk_all < max_keys ? nk_all : max_keys;
    const int lane = (int)lane_id();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const auto clamp = [](uint64_t v) { return (uint32_t)(v < 0xffffffffull ? v : 0xffffffffull); };
    for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const uint64_t first = tri_first[item];
        const int jb = ij.job_of(item);
        const fvv_grid g = jobs[jb].grid;
        const int32_t wr = (g.dims[0] + 63) / 64;
        const int64_t w0 = (int64_t)(item - ij.first_item(jb)) * kEdgeWords;   // item's first word
        const int64_t w = w0 + threadIdx.x;
        CellRows c;
        c.mixed = 0;
        if (w < fine_bitmap_words(g))
            c = cell_rows(bits + pre[jb].bit_off, w, g.dims, wr);
        uint32_t total;
        const uint32_t tri_ex = block_exclusive_sum<kBlock>(cell_triangles(c, s_tbl), scratch, &total);
        // the wave's cells, listed by word then bit
        const uint32_t n_cells = (uint32_t)__popcll(c.mixed);
        const uint32_t cell_in = wave_inclusive_sum(n_cells);
        const uint32_t cell_ex = cell_in - n_cells;
        const uint32_t wave_cells = (uint32_t)__builtin_amdgcn_readlane((int)cell_in, kWave - 1);
        const WordEdges* we = wedges + pre[jb].bit_off;
        const int64_t slab = (int64_t)wr * g.dims[1];
        const int64_t nx = g.dims[0], sz = (int64_t)g.dims[0] * g.dims[1];
        bool missing = false;
        if (c.mixed) {
#pragma unroll
            for (int m = 0; m < 4; ++m)
                s_own[m][threadIdx.x] = we[w + (m & 1) * (int64_t)wr + (m >> 1) * slab];
        }
        for (uint32_t base = 0; base < wave_cells; base += kCellRecs) {
            if (n_cells && cell_ex < base + kCellRecs && cell_ex + n_cells > base) {
                uint32_t k = cell_ex, t = tri_ex;
                for (uint64_t bm = c.mixed; bm; bm &= bm - 1, ++k) {
                    const int b = __ffsll((unsigned long long)bm) - 1;
                    const int cs = cell_pattern(c, b);
                    if (k >= base && k < base + kCellRecs)
                        s_rec[wv][k - base] = cell_rec(lane, b, cs, t);
                    t += s_tbl.count[cs];
                }
            }
            wave_lds_sync();
            const uint32_t n_here = wave_cells - base < kCellRecs ? wave_cells - base : kCellRecs;
            for (uint32_t i = lane; i < n_here; i += kWave) {
                const uint2 rec = s_rec[wv][i];
                const int src = (int)(rec.x & 63u), b = (int)((rec.x >> 6) & 63u);
                const int cs = (int)(rec.x >> 12);
                const int64_t ws = w0 + wv * kWave + src;      // the cell's word
                const int64_t row = ws / wr;
                const int32_t q = (int32_t)(ws - row * wr);
                // position of the first edge at each owner (m, dx) and the
                // x- and y-edge bits there; dx = 1 at b = 63 is the next word's bit 0
                uint32_t R[4][2], xb[4][2], yb[4][2];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const WordEdges own = s_own[m][wv * kWave + src];
                    uint64_t nex = 0, ney = 0, nez = 0;
                    uint32_t nfirst = 0;
                    if (b == 63) {
                        const WordEdges* t = we + ws + (m & 1) * (int64_t)wr + (m >> 1) * slab + 1;
                        nex = t->ex;
                        ney = t->ey;
                        nez = t->ez;
                        nfirst = t->first;
                    }
#pragma unroll
                    for (int dx = 0; dx < 2; ++dx) {
                        const bool over = dx == 1 && b == 63;
                        const uint64_t ex = over ? nex : own.ex;
                        const uint64_t ey = over ? ney : own.ey;
                        const uint64_t ez = over ? nez : own.ez;
                        const uint32_t fst = over ? nfirst : own.first;
                        const int p = over ? 0 : b + dx;
                        const uint64_t below = (1ull << p) - 1ull;
                        R[m][dx] = fst + (uint32_t)(__popcll(ex & below) + __popcll(ey & below) +
                                                    __popcll(ez & below));
                        xb[m][dx] = (uint32_t)((ex >> p) & 1u);
                        yb[m][dx] = (uint32_t)((ey >> p) & 1u);
                    }
                }
                // cell edge 4 a + u + 2 v: x-edges own (0, u, v), y-edges (u, 0, v),
                // z-edges (u, v, 0); its corners c0 and c0 + (1 << a)
                const int64_t lin0 = row * nx + 64 * (int64_t)q + b;   // corner 0
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int v = 0; v < 2; ++v) {
                            const int dx = a == 0 ? 0 : u;
                            const int dy = a == 1 ? 0 : (a == 0 ? u : v);
                            const int dz = a == 2 ? 0 : v;
                            const int m = dy + 2 * dz;
                            const uint32_t ix = R[m][dx] + (a >= 1 ? xb[m][dx] : 0u) +
                                                (a >= 2 ? yb[m][dx] : 0u);
                            const int c0 = dx + 2 * dy + 4 * dz;
                            const bool crosses = ((cs >> c0) ^ (cs >> (c0 + (1 << a)))) & 1;
                            bool bad = ix >= nk;
                            if (kVerify && crosses && !bad)
                                bad = keys[ix] !=
                                      (uint32_t)(3 * (lin0 + dx + nx * dy + sz * dz) + a);
                            missing |= crosses && bad;
                            s_pos[4 * a + u + 2 * v][threadIdx.x] = bad ? 0xffffffffu : ix;
                        }
                const int nt = s_tbl.count[cs];
                uint64_t pos = first + rec.y;
                for (int r = 0; r < nt; ++r, ++pos) {
                    if (pos >= max_tris)
                        continue;
#pragma unroll
                    for (int v = 0; v < 3; ++v)
                        tris[3 * pos + v] = s_pos[s_tbl.edge[cs][3 * r + v]][threadIdx.x];
                }
            }
            wave_lds_sync();   // the next pass rewrites this wave's records
        }
        if (missing)
            atomicOr(status, kFlagCapacity);
        if (threadIdx.x == 0) {
            if (tri_off && item == ij.first_item(jb))
                tri_off[jb] = clamp(first);
            if (item + 1 == n_items) {
                const uint64_t all = first + total;
                if (tri_off)
                    tri_off[nj] = clamp(all);
                if (n_tris)
                    *n_tris = clamp(all);
                if (all > max_tris)
                    atomicOr(status, kFlagCapacity);
            }
        }
    }
}

// Workgroups of the mesh passes: what the CUs hold at once (the write pass's
// LDS allows two per CU), or fewer when the item count is known.
static unsigned mesh_grid(const fvv_ctx* ctx, int per_cu, int64_t items_hint) {
    const int64_t full = (int64_t)ctx->n_cus * per_cu;
    return (unsigned)(items_hint > 0 && items_hint < full ? items_hint : full);
}

hipError_t launch_mesh_count(fvv_ctx* ctx, const fvv_job* jobs, const uint32_t* n_jobs_dev,
                             int64_t items_hint, hipStream_t s) {
    hipLaunchKernelGGL(mesh_count_kernel, dim3(mesh_grid(ctx, 8, items_hint)), dim3(kBlock), 0, s,
                       jobs,
                       ctx->d_prefix, n_jobs_dev, ctx->d_finebits, ctx->d_mesh_table,
                       ctx->d_tri_first, ctx->d_counter + kCounterMesh);
    return hipGetLastError();
}

hipError_t launch_mesh_write(fvv_ctx* ctx, const fvv_job* jobs, const uint32_t* n_jobs_dev,
                             const uint32_t* keys, const uint32_t* n_keys, uint32_t max_keys,
                             bool verify, uint32_t* tris, uint32_t max_tris, uint32_t* tri_off,
                             uint32_t* n_tris, int64_t items_hint, hipStream_t s) {
    auto kernel = verify ? mesh_write_kernel<true> : mesh_write_kernel<false>;
    hipLaunchKernelGGL(kernel, dim3(mesh_grid(ctx, 2, items_hint)), dim3(kBlock), 0, s, jobs,
                       ctx->d_prefix,
                       n_jobs_dev, ctx->d_finebits, ctx->d_mesh_table, ctx->d_tri_first,
                       ctx->d_word_edges, keys, n_keys, max_keys, tris, max_tris, tri_off, n_tris,
                       ctx->d_status);
    return hipGetLastError();
}

hipError_t launch_mesh(fvv_ctx* ctx, const fvv_grid& g, const uint8_t* occ, const uint32_t* keys,
                       const uint32_t* n_keys, uint32_t max_keys, uint32_t* tris,
                       uint32_t max_tris, uint32_t* n_tris, hipStream_t s) {
    fvv_job job;
    memset(&job, 0, sizeof(job));
    job.grid = g;
    const SurfaceScratch sc = surface_scratch(ctx);
    hipError_t e = launch_surface_prepare_single(sc, job, occ, s);
    if (e == hipSuccess)
        e = launch_edges(sc, ctx->d_job_single, ctx->d_counts_single + 3, nullptr, nullptr, 0,
                         nullptr, nullptr, false, true, s);
    const int64_t items = (fine_bitmap_words(g) + kEdgeWords - 1) / kEdgeWords;
    if (e == hipSuccess)
        e = launch_mesh_count(ctx, ctx->d_job_single, ctx->d_counts_single + 3, items, s);
    if (e == hipSuccess)
        e = launch_mesh_write(ctx, ctx->d_job_single, ctx->d_counts_single + 3, keys, n_keys,
                              max_keys, true, tris, max_tris, nullptr, n_tris, items, s);
    return e;
}

}  // namespace fvv
