/*
 * CPU oracle for the coarse-to-fine visual-hull path of Chen et al.,
 * "A Fast Free-viewpoint Video Synthesis Algorithm for Sports Scenes".
 *
 * TEST INFRASTRUCTURE ONLY.  This file is what the GPU path is checked
 * against; the product never calls it.  It shares no code, header, table or
 * helper with the HIP library, and is written to be read against the paper:
 * plain loops, fp32 where the method computes in fp32, the plainest exact
 * definition everywhere else.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * (-ffp-contract=off matters: every fused multiply-add below is an explicit
 * fmaf, and no other expression may be contracted into one).
 *
 * Paper sections followed:
 *   orc_carve        Sec. II-B (volumetric visual hull): a voxel is occupied iff
 *                    its projection falls inside every camera's silhouette.
 *   orc_label        Sec. II-B-2: 26-adjacency connected components, the
 *                    minimum 3-D bounding box of each, and the size filter of
 *                    Eq. (1) (read as: keep iff T_np <= N(S) <= T_nb).
 *   orc_label_bfs    the same components by breadth-first flood fill (a pin).
 *   orc_roi_fine     Sec. II-B-3: each ROI becomes its own fine volume.
 *   orc_edges        Sec. II-C: grid edges whose two endpoints differ.
 *   orc_bisect       Sec. II-C, Eq. (2)-(3): the point where an edge leaves the
 *                    hull, i.e. the first exit over all cameras, located by
 *                    bisection of the 3-D edge parameter.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ pixels */

/* Exact floor of the real quotient a/w, for w > 0.  The double quotient of two
 * floats is never rounded across an integer while |a/w| < 2^29 (their
 * difference from any integer is at least 2^-24*min(1,|a/w|), far above the
 * double's rounding error), so floor of the double quotient is exact. */
int64_t orc_floor_div(float a, float w)
{
    return (int64_t)floor((double)a / (double)w);
}

/* Pixel index of the image coordinate a/w along an axis of `dim` pixels
 * (pixel x covers [x, x+1)); -1 when the point is behind the camera (w <= 0,
 * or NaN) or outside the image. */
static int pixel_index(float a, float w, int dim)
{
    if (!(w > 0.0f))
        return -1;
    double q = (double)a / (double)w;
    if (!(q >= 0.0 && q < (double)dim))
        return -1;
    return (int)floor(q);
}

/* Silhouette bit of pixel (x, y) of camera c; bit x&31 of word x>>5 of a row. */
static int sil_bit(const uint32_t *sils, int c, int H, int wpr, int x, int y)
{
    uint32_t word = sils[((size_t)c * H + y) * wpr + (x >> 5)];
    return (int)((word >> (x & 31)) & 1u);
}

/* One world point against the cameras in index order, stopping at the first
 * camera that sees background.  *ntested counts cameras tested. */
static int point_inside(int ncam, const float *P, int W, int H, const uint32_t *sils,
                        float X, float Y, float Z, int *ntested)
{
    int wpr = (W + 31) / 32;
    for (int c = 0; c < ncam; ++c) {
        const float *p = P + 12 * c;
        float a = fmaf(p[2], Z, fmaf(p[1], Y, fmaf(p[0], X, p[3])));
        float b = fmaf(p[6], Z, fmaf(p[5], Y, fmaf(p[4], X, p[7])));
        float w = fmaf(p[10], Z, fmaf(p[9], Y, fmaf(p[8], X, p[11])));
        *ntested += 1;
        int px = pixel_index(a, w, W);
        int py = pixel_index(b, w, H);
        if (px < 0 || py < 0)
            return 0;
        if (!sil_bit(sils, c, H, wpr, px, py))
            return 0;
    }
    return 1;
}

/* World coordinate of lattice index g on one axis. */
static float lattice_coord(int32_t g, float h, float o)
{
    return fmaf((float)g, h, o);
}

/* Pack uint8 masks [n][H][W] (non-zero = foreground) into rows of 32-bit words. */
void orc_pack(int n, int W, int H, const uint8_t *masks, uint32_t *out)
{
    int wpr = (W + 31) / 32;
    memset(out, 0, (size_t)n * H * wpr * sizeof(uint32_t));
    for (int c = 0; c < n; ++c)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x)
                if (masks[((size_t)c * H + y) * W + x])
                    out[((size_t)c * H + y) * wpr + (x >> 5)] |= 1u << (x & 31);
}

/* Occupancy of every sample of the lattice {o, h, lo, n}; returns the number
 * of (voxel, camera) tests made under the index-order early exit. */
int64_t orc_carve(int ncam, const float *P, int W, int H, const uint32_t *sils,
                  const float *o, float h, const int32_t *lo, const int32_t *n, uint8_t *occ)
{
    int64_t T = 0;
#pragma omp parallel for schedule(dynamic) reduction(+ : T)
    for (int k = 0; k < n[2]; ++k) {
        float Z = lattice_coord(lo[2] + k, h, o[2]);
        for (int j = 0; j < n[1]; ++j) {
            float Y = lattice_coord(lo[1] + j, h, o[1]);
            for (int i = 0; i < n[0]; ++i) {
                float X = lattice_coord(lo[0] + i, h, o[0]);
                int nt = 0;
                size_t lin = (size_t)i + (size_t)n[0] * ((size_t)j + (size_t)n[1] * k);
                occ[lin] = (uint8_t)point_inside(ncam, P, W, H, sils, X, Y, Z, &nt);
                T += nt;
            }
        }
    }
    return T;
}

/* ------------------------------------------------------------------ labelling */

static int32_t uf_find(int32_t *parent, int32_t x)
{
    while (parent[x] != x) {
        parent[x] = parent[parent[x]];
        x = parent[x];
    }
    return x;
}

/* Link the larger root under the smaller: every tree's root is its minimum. */
static void uf_union(int32_t *parent, int32_t a, int32_t b)
{
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a < b)
        parent[b] = a;
    else if (b < a)
        parent[a] = b;
}

/*
 * 26-adjacency components of the ON samples of an n[0] x n[1] x n[2] grid
 * (x fastest), by sequential union-find over each voxel's 13 neighbours that
 * come earlier in raster order.  Components with T_np <= N(S) <= T_nb are
 * kept and numbered 1..K in ascending order of their smallest linear index;
 * the others are switched OFF in occ.  labels[v] is the number of v's kept
 * component, 0 for background and removed voxels.  rois (8 int32 per row:
 * lo[3], hi[3] inclusive grid-local indices, voxel count, smallest linear
 * index) receives min(K, max_rois) rows.  Returns K.
 */
int32_t orc_label(const int32_t *n, uint8_t *occ, int32_t *labels, uint32_t t_np,
                  uint32_t t_nb, int32_t *rois, int32_t max_rois)
{
    const int nx = n[0], ny = n[1], nz = n[2];
    const int32_t V = nx * ny * nz;
    int32_t *parent = (int32_t *)malloc((size_t)V * sizeof(int32_t));
    for (int32_t v = 0; v < V; ++v)
        parent[v] = v;

    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int32_t v = i + nx * (j + ny * k);
                if (!occ[v])
                    continue;
                for (int dk = -1; dk <= 0; ++dk)
                    for (int dj = -1; dj <= 1; ++dj)
                        for (int di = -1; di <= 1; ++di) {
                            /* the 13 neighbours that precede v in raster order */
                            if (dk == 0 && (dj > 0 || (dj == 0 && di >= 0)))
                                continue;
                            int ii = i + di, jj = j + dj, kk = k + dk;
                            if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0)
                                continue;
                            int32_t u = ii + nx * (jj + ny * kk);
                            if (occ[u])
                                uf_union(parent, v, u);
                        }
            }

    uint32_t *count = (uint32_t *)calloc((size_t)V, sizeof(uint32_t));
    int32_t *box = (int32_t *)malloc((size_t)V * 6 * sizeof(int32_t));
    int32_t *lab = (int32_t *)calloc((size_t)V, sizeof(int32_t));
    for (int32_t v = 0; v < V; ++v) {
        if (!occ[v])
            continue;
        int32_t r = uf_find(parent, v);
        int i = v % nx, j = (v / nx) % ny, k = v / (nx * ny);
        if (count[r] == 0) {
            box[6 * r + 0] = box[6 * r + 3] = i;
            box[6 * r + 1] = box[6 * r + 4] = j;
            box[6 * r + 2] = box[6 * r + 5] = k;
        }
        count[r] += 1;
        if (i < box[6 * r + 0]) box[6 * r + 0] = i;
        if (j < box[6 * r + 1]) box[6 * r + 1] = j;
        if (k < box[6 * r + 2]) box[6 * r + 2] = k;
        if (i > box[6 * r + 3]) box[6 * r + 3] = i;
        if (j > box[6 * r + 4]) box[6 * r + 4] = j;
        if (k > box[6 * r + 5]) box[6 * r + 5] = k;
    }

    int32_t K = 0;
    for (int32_t v = 0; v < V; ++v) {          /* roots in ascending index order */
        if (!occ[v] || parent[v] != v)
            continue;
        if (count[v] < t_np || count[v] > t_nb)
            continue;
        lab[v] = ++K;
        if (K <= max_rois) {
            int32_t *row = rois + 8 * (K - 1);
            for (int a = 0; a < 6; ++a)
                row[a] = box[6 * v + a];
            row[6] = (int32_t)count[v];
            row[7] = v;
        }
    }
    for (int32_t v = 0; v < V; ++v) {
        labels[v] = occ[v] ? lab[uf_find(parent, v)] : 0;
        occ[v] = (uint8_t)(labels[v] != 0);
    }
    free(parent);
    free(count);
    free(box);
    free(lab);
    return K;
}

/* Components by breadth-first flood fill from seeds met in raster order:
 * comp[v] = 1-based component number (0 = background).  Returns the count. */
int32_t orc_label_bfs(const int32_t *n, const uint8_t *occ, int32_t *comp)
{
    const int nx = n[0], ny = n[1], nz = n[2];
    const int32_t V = nx * ny * nz;
    int32_t *queue = (int32_t *)malloc((size_t)(V > 0 ? V : 1) * sizeof(int32_t));
    memset(comp, 0, (size_t)V * sizeof(int32_t));
    int32_t ncomp = 0;
    for (int32_t s = 0; s < V; ++s) {
        if (!occ[s] || comp[s])
            continue;
        comp[s] = ++ncomp;
        int32_t head = 0, tail = 0;
        queue[tail++] = s;
        while (head < tail) {
            int32_t v = queue[head++];
            int i = v % nx, j = (v / nx) % ny, k = v / (nx * ny);
            for (int dk = -1; dk <= 1; ++dk)
                for (int dj = -1; dj <= 1; ++dj)
                    for (int di = -1; di <= 1; ++di) {
                        int ii = i + di, jj = j + dj, kk = k + dk;
                        if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz)
                            continue;
                        int32_t u = ii + nx * (jj + ny * kk);
                        if (occ[u] && !comp[u]) {
                            comp[u] = ncomp;
                            queue[tail++] = u;
                        }
                    }
        }
    }
    free(queue);
    return ncomp;
}

/* ------------------------------------------------------------------ ROI lattices */

static int64_t floor_div_i64(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0)))
        q -= 1;
    return q;
}

static int64_t ceil_div_i64(int64_t a, int64_t b)
{
    return -floor_div_i64(-a, b);
}

/*
 * Fine lattice of one ROI.  All lattices share the world origin; voxel sizes
 * are integer micrometres.  A coarse box [a, b] (grid-local, inclusive) is
 * dilated by one coarse cell, mapped to fine global indices
 * [floor((A-1) hc / hf), ceil((B+1) hc / hf)] with A, B the global coarse
 * indices, and clamped to the fine samples that lie within the coarse
 * lattice's extent.  Outputs the fine lattice's first global index and size.
 */
void orc_roi_fine(const int32_t *coarse_lo, const int32_t *coarse_n, int64_t hc_um,
                  int64_t hf_um, const int32_t *box_lo, const int32_t *box_hi,
                  int32_t *fine_lo, int32_t *fine_n)
{
    for (int a = 0; a < 3; ++a) {
        int64_t A = (int64_t)coarse_lo[a] + box_lo[a] - 1;
        int64_t B = (int64_t)coarse_lo[a] + box_hi[a] + 1;
        int64_t f0 = floor_div_i64(A * hc_um, hf_um);
        int64_t f1 = ceil_div_i64(B * hc_um, hf_um);
        int64_t fmin = ceil_div_i64((int64_t)coarse_lo[a] * hc_um, hf_um);
        int64_t fmax = floor_div_i64(((int64_t)coarse_lo[a] + coarse_n[a] - 1) * hc_um, hf_um);
        if (f0 < fmin) f0 = fmin;
        if (f1 > fmax) f1 = fmax;
        fine_lo[a] = (int32_t)f0;
        fine_n[a] = (int32_t)(f1 - f0 + 1);
    }
}

/* ------------------------------------------------------------------ surface */

/* Keys 3*lin(p)+axis of every lattice edge (p, p+e_axis) inside the grid whose
 * endpoints differ, ascending.  Writes at most max_keys; returns the count. */
int64_t orc_edges(const int32_t *n, const uint8_t *occ, uint32_t *keys, int64_t max_keys)
{
    const int64_t nx = n[0], ny = n[1], nz = n[2];
    int64_t E = 0;
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t lin = i + nx * (j + ny * k);
                int inb[3] = {i + 1 < nx, j + 1 < ny, k + 1 < nz};
                int64_t stride[3] = {1, nx, nx * ny};
                for (int a = 0; a < 3; ++a) {
                    if (!inb[a])
                        continue;
                    if ((occ[lin] != 0) != (occ[lin + stride[a]] != 0)) {
                        if (E < max_keys)
                            keys[E] = (uint32_t)(3 * lin + a);
                        ++E;
                    }
                }
            }
    return E;
}

/*
 * Where each crossing edge leaves the hull.  The edge runs from its ON
 * endpoint (parameter 0) to its OFF endpoint (parameter 1) along one lattice
 * axis.  Each of `steps` bisection steps tests the midpoint m of the current
 * bracket [lo, hi] against all cameras (the occupancy test of orc_carve): an
 * inside midpoint moves lo up, an outside one moves hi down.  This locates the
 * first exit over all cameras, the minimum over cameras of Eq. (3), at the
 * resolution 2^-steps.  Output: t* = (lo+hi)/2 and the world point there,
 * with the axis coordinate computed as fmaf(g_on + d*t*, h, o) (d = +1 or -1
 * toward the OFF endpoint) and the other two coordinates as lattice values.
 */
int64_t orc_bisect(int ncam, const float *P, int W, int H, const uint32_t *sils,
                   const float *o, float h, const int32_t *lo, const int32_t *n,
                   const uint8_t *occ, const uint32_t *keys, int64_t E, int steps,
                   float *xyz, float *tstar)
{
    int64_t tests = 0;
#pragma omp parallel for schedule(static) reduction(+ : tests)
    for (int64_t e = 0; e < E; ++e) {
        int64_t lin = keys[e] / 3;
        int axis = (int)(keys[e] % 3);
        int64_t i = lin % n[0], j = (lin / n[0]) % n[1], k = lin / ((int64_t)n[0] * n[1]);
        int64_t stride = axis == 0 ? 1 : (axis == 1 ? n[0] : (int64_t)n[0] * n[1]);
        int32_t g[3] = {lo[0] + (int32_t)i, lo[1] + (int32_t)j, lo[2] + (int32_t)k};
        int p_on = occ[lin] != 0;
        int q_on = occ[lin + stride] != 0;
        (void)q_on;
        int32_t g_on = p_on ? g[axis] : g[axis] + 1;
        float d = p_on ? 1.0f : -1.0f;

        float c[3];
        for (int a = 0; a < 3; ++a)
            c[a] = lattice_coord(g[a], h, o[a]);

        float tlo = 0.0f, thi = 1.0f;
        for (int s = 0; s < steps; ++s) {
            float m = 0.5f * (tlo + thi);
            float q = (float)g_on + d * m;
            c[axis] = fmaf(q, h, o[axis]);
            int nt = 0;
            if (point_inside(ncam, P, W, H, sils, c[0], c[1], c[2], &nt))
                tlo = m;
            else
                thi = m;
            tests += nt;
        }
        float t = 0.5f * (tlo + thi);
        float q = (float)g_on + d * t;
        c[axis] = fmaf(q, h, o[axis]);
        xyz[3 * e + 0] = c[0];
        xyz[3 * e + 1] = c[1];
        xyz[3 * e + 2] = c[2];
        tstar[e] = t;
    }
    return tests;
}

/* Single world point against all cameras (for checks of the occupancy test). */
int32_t orc_point_inside(int ncam, const float *P, int W, int H, const uint32_t *sils,
                         float X, float Y, float Z)
{
    int nt = 0;
    return point_inside(ncam, P, W, H, sils, X, Y, Z, &nt);
}

/* Threads the OpenMP loops above use. */
#ifdef _OPENMP
#include <omp.h>
#endif
int32_t orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
