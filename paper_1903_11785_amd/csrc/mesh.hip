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
// A work item is kMeshItem consecutive cells (linear order over the
// (nx-1) x (ny-1) x (nz-1) cells, x fastest), kMeshCellsPerThread per thread.
// The count pass sums each item's triangles; the write pass adds the counts of
// the earlier items, scans its threads and writes each thread's cells in order.
// Cell indices are 32-bit (fvv_mesh bounds the lattice).
constexpr int kMeshCellsPerThread = 16;
constexpr int kMeshItem = kBlock * kMeshCellsPerThread;

struct CellGeom {
    uint32_t cx, cy, cells;
    int64_t sy, sz;
};

// Corner pattern of cell c and its first sample's linear index.
__device__ __forceinline__ int cell_case(const uint8_t* __restrict__ occ, uint32_t c,
                                         const CellGeom& cg, int64_t& base) {
    const uint32_t r = c / cg.cx, i = c - r * cg.cx;
    const uint32_t k = r / cg.cy, j = r - k * cg.cy;
    base = (int64_t)i + cg.sy * j + cg.sz * k;
    const uint8_t* o = occ + base;
    int cs = (o[0] != 0) | (o[1] != 0) << 1 | (o[cg.sy] != 0) << 2 | (o[cg.sy + 1] != 0) << 3;
    o += cg.sz;
    cs |= (o[0] != 0) << 4 | (o[1] != 0) << 5 | (o[cg.sy] != 0) << 6 | (o[cg.sy + 1] != 0) << 7;
    return cs;
}

__device__ __forceinline__ CellGeom cell_geom(const fvv_grid& g) {
    CellGeom cg;
    cg.cx = (uint32_t)(g.dims[0] - 1);
    cg.cy = (uint32_t)(g.dims[1] - 1);
    cg.cells = cg.cx * cg.cy * (uint32_t)(g.dims[2] - 1);
    cg.sy = g.dims[0];
    cg.sz = (int64_t)g.dims[0] * g.dims[1];
    return cg;
}

__global__ __launch_bounds__(kBlock) void mesh_count_kernel(const fvv_grid g,
                                                            const uint8_t* __restrict__ occ,
                                                            const MeshTable* __restrict__ tbl,
                                                            uint32_t* __restrict__ item_cnt) {
    __shared__ uint32_t scratch[kBlock / kWave];
    const CellGeom cg = cell_geom(g);
    const uint32_t items = (cg.cells + kMeshItem - 1) / kMeshItem;
    for (uint32_t it = blockIdx.x; it < items; it += gridDim.x) {
        uint32_t n = 0;
        const uint32_t c0 = it * kMeshItem + threadIdx.x * kMeshCellsPerThread;
        for (int q = 0; q < kMeshCellsPerThread; ++q)
            if (c0 + q < cg.cells) {
                int64_t base;
                n += tbl->count[cell_case(occ, c0 + q, cg, base)];
            }
        uint32_t tot;
        block_exclusive_sum<kBlock>(n, scratch, &tot);
        if (threadIdx.x == 0)
            item_cnt[it] = tot;
        __syncthreads();
    }
}

// Index of `key` in keys[0, n) (ascending), or -1.
__device__ __forceinline__ int64_t key_index(const uint32_t* __restrict__ keys, int64_t n,
                                             uint32_t key) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < n && keys[lo] == key) ? lo : -1;
}

__global__ __launch_bounds__(kBlock) void mesh_write_kernel(
    const fvv_grid g, const uint8_t* __restrict__ occ, const MeshTable* __restrict__ tbl,
    const uint32_t* __restrict__ item_cnt, const uint32_t* __restrict__ keys,
    const uint32_t* __restrict__ n_keys_p, uint32_t max_keys, uint32_t* __restrict__ tris,
    uint32_t max_tris, uint32_t* __restrict__ n_tris, uint32_t* __restrict__ status) {
    __shared__ uint32_t scratch[kBlock / kWave];
    __shared__ uint32_t s_before;
    const CellGeom cg = cell_geom(g);
    const uint32_t items = (cg.cells + kMeshItem - 1) / kMeshItem;
    const uint32_t nk_all = *n_keys_p;
    const int64_t nk = nk_all < max_keys ? nk_all : max_keys;
    for (uint32_t it = blockIdx.x; it < items; it += gridDim.x) {
        // triangles of all earlier work items
        uint32_t part = 0;
        for (uint32_t p = threadIdx.x; p < it; p += kBlock)
            part += item_cnt[p];
        uint32_t before;
        block_exclusive_sum<kBlock>(part, scratch, &before);
        if (threadIdx.x == 0)
            s_before = before;
        __syncthreads();
        const uint32_t item_base = s_before;
        // this thread's cells follow the lower threads' triangles
        const uint32_t c0 = it * kMeshItem + threadIdx.x * kMeshCellsPerThread;
        uint32_t n = 0;
        for (int q = 0; q < kMeshCellsPerThread; ++q)
            if (c0 + q < cg.cells) {
                int64_t base;
                n += tbl->count[cell_case(occ, c0 + q, cg, base)];
            }
        uint32_t tot;
        uint32_t pos = item_base + block_exclusive_sum<kBlock>(n, scratch, &tot);
        bool missing = false;
        for (int q = 0; q < kMeshCellsPerThread && n; ++q) {
            if (c0 + q >= cg.cells)
                break;
            int64_t base;
            const int cs = cell_case(occ, c0 + q, cg, base);
            const int nt = tbl->count[cs];
            for (int r = 0; r < nt; ++r, ++pos) {
                if (pos >= max_tris)
                    continue;
#pragma unroll
                for (int v = 0; v < 3; ++v) {
                    const int e = tbl->edge[cs][3 * r + v];
                    const int a = e >> 2, u = e & 1, w = (e >> 1) & 1;
                    // the edge's first sample: 0 on axis a, (u, w) on the other two
                    const int dx = a == 0 ? 0 : u;
                    const int dy = a == 1 ? 0 : (a == 0 ? u : w);
                    const int dz = a == 2 ? 0 : w;
                    const int64_t lin = base + dx + cg.sy * dy + cg.sz * dz;
                    const int64_t ix = key_index(keys, nk, (uint32_t)(3 * lin + a));
                    missing |= ix < 0;
                    tris[3 * (int64_t)pos + v] = ix < 0 ? 0xffffffffu : (uint32_t)ix;
                }
            }
        }
        if (missing)
            atomicOr(status, kFlagCapacity);
        if (it == items - 1 && threadIdx.x == kBlock - 1) {
            const uint32_t all = item_base + tot;
            *n_tris = all;
            if (all > max_tris)
                atomicOr(status, kFlagCapacity);
        }
        __syncthreads();
    }
}

__global__ void mesh_zero_kernel(uint32_t* __restrict__ n_tris) { *n_tris = 0u; }

hipError_t launch_mesh(fvv_ctx* ctx, const fvv_grid& g, const uint8_t* occ, const uint32_t* keys,
                       const uint32_t* n_keys, uint32_t max_keys, uint32_t* tris,
                       uint32_t max_tris, uint32_t* n_tris, hipStream_t s) {
    const int64_t cells = (int64_t)(g.dims[0] - 1) * (g.dims[1] - 1) * (g.dims[2] - 1);
    if (cells <= 0) {
        hipLaunchKernelGGL(mesh_zero_kernel, dim3(1), dim3(1), 0, s, n_tris);
        return hipGetLastError();
    }
    const int64_t items = (cells + kMeshItem - 1) / kMeshItem;
    const unsigned blocks = (unsigned)(items < (int64_t)ctx->n_cus * 8 ? items : ctx->n_cus * 8);
    hipLaunchKernelGGL(mesh_count_kernel, dim3(blocks), dim3(kBlock), 0, s, g, occ,
                       ctx->d_mesh_table, ctx->d_item_cnt);
    hipLaunchKernelGGL(mesh_write_kernel, dim3(blocks), dim3(kBlock), 0, s, g, occ,
                       ctx->d_mesh_table, ctx->d_item_cnt, keys, n_keys, max_keys, tris, max_tris,
                       n_tris, ctx->d_status);
    return hipGetLastError();
}

int64_t mesh_items(const fvv_grid& g) {
    const int64_t cells = (int64_t)(g.dims[0] - 1) * (g.dims[1] - 1) * (g.dims[2] - 1);
    return cells <= 0 ? 0 : (cells + kMeshItem - 1) / kMeshItem;
}

}  // namespace fvv
