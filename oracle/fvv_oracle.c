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
 *   orc_isovalue     Sec. II-C, Eq. (2)-(3) as the paper computes them: per
 *                    camera the last foreground pixel of the Bresenham line
 *                    from P_on to P_off, the image-space ratio of Eq. (2),
 *                    the minimum over cameras of Eq. (3).
 *   orc_mesh         Sec. II-C: marching-cubes triangles over the cells.
 *   orc_depth        Sec. II-D-1, Eq. (4): per camera, the minimum over the
 *                    triangles covering a pixel of their distance.
 *   orc_visibility   Sec. II-D-2: a triangle is occluded in a camera when its
 *                    distance exceeds the depth image by more than T_v.
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
 * The world point at parameter t of a crossing edge (Sec. II-C).  The edge
 * key 3*lin+axis names the lattice edge from sample lin to its neighbour
 * along `axis`; parameter 0 is its ON endpoint (the occupied one), 1 its OFF
 * endpoint.  The axis coordinate is fmaf(g_on + d*t, h, o) with d = +1 or -1
 * toward the OFF endpoint; the other two are lattice values.
 */
static void edge_point(const float *o, float h, const int32_t *lo, const int32_t *n,
                       const uint8_t *occ, uint32_t key, float t, float *xyz)
{
    int64_t lin = key / 3;
    int axis = (int)(key % 3);
    int64_t i = lin % n[0], j = (lin / n[0]) % n[1], k = lin / ((int64_t)n[0] * n[1]);
    int32_t g[3] = {lo[0] + (int32_t)i, lo[1] + (int32_t)j, lo[2] + (int32_t)k};
    int p_on = occ[lin] != 0;
    int32_t g_on = p_on ? g[axis] : g[axis] + 1;
    float d = p_on ? 1.0f : -1.0f;
    for (int a = 0; a < 3; ++a)
        xyz[a] = lattice_coord(g[a], h, o[a]);
    float q = (float)g_on + d * t;
    xyz[axis] = fmaf(q, h, o[axis]);
}

/*
 * Where each crossing edge leaves the hull.  Each of `steps` bisection steps
 * tests the point at the midpoint m of the current bracket [lo, hi] of the
 * edge parameter (edge_point) against all cameras (the occupancy test of
 * orc_carve): an inside midpoint moves lo up, an outside one moves hi down.
 * This locates the first exit over all cameras, the minimum over cameras of
 * Eq. (3), at the resolution 2^-steps.  Output: t* = (lo+hi)/2 and the world
 * point there.
 */
int64_t orc_bisect(int ncam, const float *P, int W, int H, const uint32_t *sils,
                   const float *o, float h, const int32_t *lo, const int32_t *n,
                   const uint8_t *occ, const uint32_t *keys, int64_t E, int steps,
                   float *xyz, float *tstar)
{
    int64_t tests = 0;
#pragma omp parallel for schedule(static) reduction(+ : tests)
    for (int64_t e = 0; e < E; ++e) {
        float c[3];
        float tlo = 0.0f, thi = 1.0f;
        for (int s = 0; s < steps; ++s) {
            float m = 0.5f * (tlo + thi);
            edge_point(o, h, lo, n, occ, keys[e], m, c);
            int nt = 0;
            if (point_inside(ncam, P, W, H, sils, c[0], c[1], c[2], &nt))
                tlo = m;
            else
                thi = m;
            tests += nt;
        }
        float t = 0.5f * (tlo + thi);
        edge_point(o, h, lo, n, occ, keys[e], t, xyz + 3 * e);
        tstar[e] = t;
    }
    return tests;
}

/* The point of edge `key` at parameter t, as orc_bisect forms it (for checks
 * of the bisection's brackets). */
void orc_edge_point(const float *o, float h, const int32_t *lo, const int32_t *n,
                    const uint8_t *occ, uint32_t key, float t, float *xyz)
{
    edge_point(o, h, lo, n, occ, key, t, xyz);
}

/* Single world point against all cameras (for checks of the occupancy test). */
int32_t orc_point_inside(int ncam, const float *P, int W, int H, const uint32_t *sils,
                         float X, float Y, float Z)
{
    int nt = 0;
    return point_inside(ncam, P, W, H, sils, X, Y, Z, &nt);
}

/* ------------------------------------------------------------------ isovalue (Bresenham)
 *
 * The paper's own isovalue of a crossing edge (Sec. II-C, Eq. (2) and (3)),
 * with the readings the paper leaves open fixed as follows.  In camera i the
 * edge's ends project to the pixels P_on (the occupied end's: inside the
 * image and foreground, since that sample is occupied) and P_off (the exact
 * floor of its projection, clamped to [-8, dim + 8] on each axis).  The line
 * of pixels from P_on to P_off is traced with Bresenham's integer algorithm
 * (all octants: the error term starts at dx - dy and each step moves along x
 * when twice the error is at least -dy, along y when it is at most dx).  P_i
 * is the last pixel before the first one that is background or outside the
 * image, and Eq. (2) gives lambda_i = |P_i - P_on| / |P_off - P_on|; a line
 * that is foreground to its end gives lambda_i = 1, and a camera that sees
 * either end behind it (w <= 0) gives lambda_i = 0.  lambda_i^2 is taken as
 * the double quotient of the two integer squared lengths; Eq. (3)'s minimum is
 * taken over those, and lambda = (float)sqrt(min).
 */

/* lambda_i^2 of one camera for the pixel line (x0, y0) -> (x1, y1) over the
 * silhouette rows `sil` ([H][wpr] words).  A start pixel that is not
 * foreground gives 0. */
static double line_lambda2(const uint32_t *sil, int W, int H, int wpr, int x0, int y0, int x1,
                           int y1)
{
    const int fg0 = x0 >= 0 && y0 >= 0 && x0 < W && y0 < H &&
                    ((sil[(size_t)y0 * wpr + (x0 >> 5)] >> (x0 & 31)) & 1u);
    if (!fg0)
        return 0.0;
    const int dx = abs(x1 - x0), dy = abs(y1 - y0);
    const int sx = x0 < x1 ? 1 : -1, sy = y0 < y1 ? 1 : -1;
    int err = dx - dy;
    int x = x0, y = y0, last_x = x0, last_y = y0;
    while (x != x1 || y != y1) {
        const int e2 = 2 * err;
        if (e2 >= -dy) {
            err -= dy;
            x += sx;
        }
        if (e2 <= dx) {
            err += dx;
            y += sy;
        }
        const int fg = x >= 0 && y >= 0 && x < W && y < H &&
                       ((sil[(size_t)y * wpr + (x >> 5)] >> (x & 31)) & 1u);
        if (!fg) {
            const int64_t ax = last_x - x0, ay = last_y - y0;
            const int64_t bx = x1 - x0, by = y1 - y0;
            return (double)(ax * ax + ay * ay) / (double)(bx * bx + by * by);
        }
        last_x = x;
        last_y = y;
    }
    return 1.0;
}

double orc_line_lambda2(const uint32_t *sil, int W, int H, int x0, int y0, int x1, int y1)
{
    return line_lambda2(sil, W, H, (W + 31) / 32, x0, y0, x1, y1);
}

/* Pixel index of the quotient a/w on one axis for the line's far end: the
 * exact floor, clamped to [-8, dim + 8]. */
static int far_pixel(float a, float w, int dim)
{
    double q = floor((double)a / (double)w);
    if (q < -8.0)
        q = -8.0;
    if (q > (double)dim + 8.0)
        q = (double)dim + 8.0;
    return (int)q;
}

void orc_isovalue(int ncam, const float *P, int W, int H, const uint32_t *sils, const float *o,
                  float h, const int32_t *lo, const int32_t *n, const uint8_t *occ,
                  const uint32_t *keys, int64_t E, float *lambda, float *xyz)
{
    const int wpr = (W + 31) / 32;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        const int64_t lin = keys[e] / 3;
        const int axis = (int)(keys[e] % 3);
        const int64_t i = lin % n[0], j = (lin / n[0]) % n[1], k = lin / ((int64_t)n[0] * n[1]);
        const int64_t stride = axis == 0 ? 1 : (axis == 1 ? n[0] : (int64_t)n[0] * n[1]);
        const int32_t g[3] = {lo[0] + (int32_t)i, lo[1] + (int32_t)j, lo[2] + (int32_t)k};
        const int p_on = occ[lin] != 0;
        (void)stride;
        const int32_t g_on = p_on ? g[axis] : g[axis] + 1;
        const int32_t g_off = p_on ? g[axis] + 1 : g[axis];
        const float d = p_on ? 1.0f : -1.0f;
        float X_on[3], X_off[3];
        for (int a = 0; a < 3; ++a)
            X_on[a] = X_off[a] = lattice_coord(g[a], h, o[a]);
        X_on[axis] = lattice_coord(g_on, h, o[axis]);
        X_off[axis] = lattice_coord(g_off, h, o[axis]);

        double best = 1.0;
        for (int c = 0; c < ncam; ++c) {
            const float *p = P + 12 * c;
            const float *X = X_on;
            const float a0 = fmaf(p[2], X[2], fmaf(p[1], X[1], fmaf(p[0], X[0], p[3])));
            const float b0 = fmaf(p[6], X[2], fmaf(p[5], X[1], fmaf(p[4], X[0], p[7])));
            const float w0 = fmaf(p[10], X[2], fmaf(p[9], X[1], fmaf(p[8], X[0], p[11])));
            X = X_off;
            const float a1 = fmaf(p[2], X[2], fmaf(p[1], X[1], fmaf(p[0], X[0], p[3])));
            const float b1 = fmaf(p[6], X[2], fmaf(p[5], X[1], fmaf(p[4], X[0], p[7])));
            const float w1 = fmaf(p[10], X[2], fmaf(p[9], X[1], fmaf(p[8], X[0], p[11])));
            double l2;
            if (!(w0 > 0.0f) || !(w1 > 0.0f))
                l2 = 0.0;
            else
                l2 = line_lambda2(sils + (size_t)c * H * wpr, W, H, wpr, far_pixel(a0, w0, W),
                                  far_pixel(b0, w0, H), far_pixel(a1, w1, W),
                                  far_pixel(b1, w1, H));
            if (l2 < best)
                best = l2;
        }
        const float lam = (float)sqrt(best);
        lambda[e] = lam;
        if (xyz) {
            float c3[3];
            for (int a = 0; a < 3; ++a)
                c3[a] = X_on[a];
            c3[axis] = fmaf((float)g_on + d * lam, h, o[axis]);
            for (int a = 0; a < 3; ++a)
                xyz[3 * e + a] = c3[a];
        }
    }
}

/* ------------------------------------------------------------------ depth and visibility
 *
 * Sec. II-D.  Readings of what the paper leaves open:
 *   - a triangle's distance is the camera-plane distance (the projection's
 *     third row, w) of its centroid G = ((v0 + v1) + v2) / 3, per component
 *     in fp32: one value per (triangle, camera);
 *   - the 2-D triangle has the vertices (a/w, b/w) of the three projections
 *     (IEEE fp32 division); it covers pixel (x, y) when the pixel centre
 *     (x + 0.5, y + 0.5) lies on the same side of its three edges, i.e. the
 *     three edge functions (x1 - x0)(py - y0) - (y1 - y0)(px - x0), evaluated
 *     in fp32 in that order, are all >= 0 or all <= 0; triangles with a vertex
 *     at w <= 0, or of zero area (the first edge's function at the third
 *     vertex is 0), cover nothing;
 *   - Eq. (4): the depth image holds the minimum covering distance, +inf
 *     where nothing covers the pixel; a triangle whose centroid distance is
 *     not positive covers nothing;
 *   - a triangle naming a vertex past the vertex count (such as the mesh's
 *     0xffffffff for a missing vertex) covers nothing and is invisible;
 *   - visibility: the centroid's projection (a_G/w_G, b_G/w_G) falls in pixel
 *     p (floor of each coordinate); the triangle is visible in the camera when
 *     w_G > 0, p lies inside the image and d - depth[p] <= T_v (fp32).
 * Triangles index a vertex array of exit points (xyz).
 */

/* Projection rows of camera P at X: a, b, w (the occupancy test's order). */
static void project3(const float *p, const float *X, float *a, float *b, float *w)
{
    *a = fmaf(p[2], X[2], fmaf(p[1], X[1], fmaf(p[0], X[0], p[3])));
    *b = fmaf(p[6], X[2], fmaf(p[5], X[1], fmaf(p[4], X[0], p[7])));
    *w = fmaf(p[10], X[2], fmaf(p[9], X[1], fmaf(p[8], X[0], p[11])));
}

/* Camera-plane distance of the triangle's centroid and its projection. */
static void triangle_centroid(const float *p, const float *xyz, const uint32_t *t, float *u,
                              float *v, float *w)
{
    float G[3], a, b;
    for (int k = 0; k < 3; ++k)
        G[k] = ((xyz[3 * (size_t)t[0] + k] + xyz[3 * (size_t)t[1] + k]) +
                xyz[3 * (size_t)t[2] + k]) / 3.0f;
    project3(p, G, &a, &b, w);
    *u = a / *w;
    *v = b / *w;
}

static float edge_fn(float x0, float y0, float x1, float y1, float px, float py)
{
    return (x1 - x0) * (py - y0) - (y1 - y0) * (px - x0);
}

void orc_depth(int ncam, const float *P, int W, int H, const float *xyz, int64_t n_vertices,
               const uint32_t *tris, int64_t T, float *depth)
{
    const size_t npx = (size_t)W * H;
#pragma omp parallel for schedule(static)
    for (int c = 0; c < ncam; ++c) {
        float *D = depth + (size_t)c * npx;
        for (size_t q = 0; q < npx; ++q)
            D[q] = INFINITY;
        const float *p = P + 12 * c;
        for (int64_t m = 0; m < T; ++m) {
            const uint32_t *t = tris + 3 * m;
            if (t[0] >= n_vertices || t[1] >= n_vertices || t[2] >= n_vertices)
                continue;
            float u[3], v[3], w[3];
            int front = 1;
            for (int k = 0; k < 3; ++k) {
                float a, b;
                project3(p, xyz + 3 * (size_t)t[k], &a, &b, &w[k]);
                if (!(w[k] > 0.0f))
                    front = 0;
                u[k] = a / w[k];
                v[k] = b / w[k];
            }
            if (!front)
                continue;
            if (edge_fn(u[0], v[0], u[1], v[1], u[2], v[2]) == 0.0f)
                continue;                       /* zero area */
            float gu, gv, d;
            triangle_centroid(p, xyz, t, &gu, &gv, &d);
            (void)gu;
            (void)gv;
            if (!(d > 0.0f))
                continue;
            /* pixels whose centres could be inside (the edge test decides) */
            float lo_u = fminf(u[0], fminf(u[1], u[2])), hi_u = fmaxf(u[0], fmaxf(u[1], u[2]));
            float lo_v = fminf(v[0], fminf(v[1], v[2])), hi_v = fmaxf(v[0], fmaxf(v[1], v[2]));
            if (!(hi_u >= 0.0f && hi_v >= 0.0f && lo_u < (float)W && lo_v < (float)H))
                continue;
            const int x0 = lo_u < 0.0f ? 0 : (int)lo_u;
            const int y0 = lo_v < 0.0f ? 0 : (int)lo_v;
            const int x1 = hi_u >= (float)(W - 1) ? W - 1 : (int)hi_u;
            const int y1 = hi_v >= (float)(H - 1) ? H - 1 : (int)hi_v;
            for (int y = y0; y <= y1; ++y)
                for (int x = x0; x <= x1; ++x) {
                    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
                    const float e0 = edge_fn(u[0], v[0], u[1], v[1], px, py);
                    const float e1 = edge_fn(u[1], v[1], u[2], v[2], px, py);
                    const float e2 = edge_fn(u[2], v[2], u[0], v[0], px, py);
                    const int in = (e0 >= 0.0f && e1 >= 0.0f && e2 >= 0.0f) ||
                                   (e0 <= 0.0f && e1 <= 0.0f && e2 <= 0.0f);
                    if (in && d < D[(size_t)y * W + x])
                        D[(size_t)y * W + x] = d;
                }
        }
    }
}

void orc_visibility(int ncam, const float *P, int W, int H, const float *xyz,
                    int64_t n_vertices, const uint32_t *tris, int64_t T, const float *depth,
                    float t_v, uint32_t *vis)
{
    const size_t npx = (size_t)W * H;
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < T; ++m) {
        uint32_t mask = 0;
        const uint32_t *t = tris + 3 * m;
        if (t[0] >= n_vertices || t[1] >= n_vertices || t[2] >= n_vertices) {
            vis[m] = 0;
            continue;
        }
        for (int c = 0; c < ncam; ++c) {
            float u, v, d;
            triangle_centroid(P + 12 * c, xyz, tris + 3 * m, &u, &v, &d);
            if (!(d > 0.0f))
                continue;
            const float fx = floorf(u), fy = floorf(v);
            if (!(fx >= 0.0f && fy >= 0.0f && fx < (float)W && fy < (float)H))
                continue;
            const float D = depth[(size_t)c * npx + (size_t)fy * W + (size_t)fx];
            if (d - D <= t_v)
                mask |= 1u << c;
        }
        vis[m] = mask;
    }
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

/* Sets the threads later parallel loops use (n >= 1); returns the previous count. */
int32_t orc_set_threads(int32_t n)
{
#ifdef _OPENMP
    int32_t prev = omp_get_max_threads();
    if (n >= 1)
        omp_set_num_threads(n);
    return prev;
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------ mesh */

/*
 * Triangles of the isosurface over the cells of one lattice (Sec. II-C: once
 * every crossing edge has its vertex, the surface follows the marching-cubes
 * configurations and is expressed as triangles).  A cell's surface crosses
 * exactly its edges whose two samples differ, one vertex per crossing edge.
 * The paper gives no configuration table, so the configurations are fixed by
 * a face rule, evaluated here cell by cell:
 *   - on each cell face, the crossing edges of the face are joined in pairs by
 *     segments: two crossing edges by one segment; four (two diagonal inside
 *     corners) by two segments, each cutting off one inside corner;
 *   - a segment runs from one crossing edge to the other so that, seen from
 *     outside the cell, the inside part of the face lies on its right;
 *   - the segments chain into closed loops (each crossing edge lies on two
 *     faces).  Each loop is cut into a fan of triangles (v0, v_i, v_i+1),
 *     facing away from the occupied corners, from the apex v0: the first
 *     vertex, in loop order from the smallest cell-edge number, that lies on
 *     no face the loop crosses twice (a loop can cross a face with four
 *     crossing edges twice; a fan diagonal between two vertices of one face
 *     would lie in that face, where the neighbouring cell may put one too).
 * Cell corners: b = dx + 2 dy + 4 dz.  Cell edges: 4 a + u + 2 v along axis a,
 * with (u, v) the corner coordinates on the other two axes in increasing axis
 * order.  Triangles are listed by cell in linear order (x fastest), loops by
 * their smallest edge, with vertices as indices into `keys` (the lattice's
 * crossing edges, ascending).  Writes at most max_tris triangles; returns
 * the count, or -1 if a crossing edge is missing from `keys`.
 */
static void cell_edge_ends(int e, int c0[3], int c1[3])
{
    const int a = e / 4, u = e & 1, v = (e >> 1) & 1;
    const int o1 = a == 0 ? 1 : 0, o2 = a == 2 ? 1 : 2;   /* the other axes, increasing */
    c0[a] = 0;
    c1[a] = 1;
    c0[o1] = c1[o1] = u;
    c0[o2] = c1[o2] = v;
}

/* next[e] = the edge a segment leads to from crossing edge e, or -1. */
static void cell_segments(const int inside[8], int next[12])
{
    for (int e = 0; e < 12; ++e)
        next[e] = -1;
    for (int a = 0; a < 3; ++a)
        for (int s = 0; s < 2; ++s) {
            /* the face's edges and their crossings */
            int fe[4], nf = 0;
            for (int e = 0; e < 12; ++e) {
                int c0[3], c1[3];
                cell_edge_ends(e, c0, c1);
                if (e / 4 != a && c0[a] == s)
                    fe[nf++] = e;
            }
            int cross[4], nc = 0;
            for (int q = 0; q < 4; ++q) {
                int c0[3], c1[3];
                cell_edge_ends(fe[q], c0, c1);
                const int b0 = c0[0] + 2 * c0[1] + 4 * c0[2], b1 = c1[0] + 2 * c1[1] + 4 * c1[2];
                if (inside[b0] != inside[b1])
                    cross[nc++] = fe[q];
            }
            if (nc == 0)
                continue;
            /* pairs of crossing edges and an inside corner for each pair */
            int pa[2], pb[2], pin[2][3], np = 0;
            if (nc == 2) {
                pa[0] = cross[0];
                pb[0] = cross[1];
                int found = 0;
                for (int b = 0; b < 8 && !found; ++b) {
                    const int c[3] = {b & 1, (b >> 1) & 1, (b >> 2) & 1};
                    if (c[a] == s && inside[b]) {
                        for (int d = 0; d < 3; ++d)
                            pin[0][d] = c[d];
                        found = 1;
                    }
                }
                np = 1;
            } else { /* four: cut off each inside corner of the face */
                for (int b = 0; b < 8; ++b) {
                    const int c[3] = {b & 1, (b >> 1) & 1, (b >> 2) & 1};
                    if (c[a] != s || !inside[b])
                        continue;
                    int m = 0, two[2];
                    for (int q = 0; q < 4; ++q) {
                        int c0[3], c1[3];
                        cell_edge_ends(cross[q], c0, c1);
                        int at0 = 1, at1 = 1;
                        for (int d = 0; d < 3; ++d) {
                            at0 &= c0[d] == c[d];
                            at1 &= c1[d] == c[d];
                        }
                        if (at0 || at1)
                            two[m++] = cross[q];
                    }
                    pa[np] = two[0];
                    pb[np] = two[1];
                    for (int d = 0; d < 3; ++d)
                        pin[np][d] = c[d];
                    ++np;
                }
            }
            /* orientation: with doubled coordinates, inside on the right seen
             * from outside means ((M2 - M1) x (P - M1)) . n < 0, n = the face's
             * outward normal */
            for (int q = 0; q < np; ++q) {
                int a0[3], a1[3], b0[3], b1[3];
                cell_edge_ends(pa[q], a0, a1);
                cell_edge_ends(pb[q], b0, b1);
                long M1[3], M2[3], P[3];
                for (int d = 0; d < 3; ++d) {
                    M1[d] = a0[d] + a1[d];
                    M2[d] = b0[d] + b1[d];
                    P[d] = 2 * pin[q][d];
                }
                const long u[3] = {M2[0] - M1[0], M2[1] - M1[1], M2[2] - M1[2]};
                const long w[3] = {P[0] - M1[0], P[1] - M1[1], P[2] - M1[2]};
                const long cr[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2],
                                    u[0] * w[1] - u[1] * w[0]};
                const long dot = cr[a] * (s ? 1 : -1);
                if (dot < 0)
                    next[pa[q]] = pb[q];
                else
                    next[pb[q]] = pa[q];
            }
        }
}

/* The two faces (2 a + s: axis a, side s) cell edge e lies on. */
static void edge_faces(int e, int f[2])
{
    int c0[3], c1[3];
    cell_edge_ends(e, c0, c1);
    int m = 0;
    for (int a = 0; a < 3; ++a)
        if (a != e / 4)
            f[m++] = 2 * a + c0[a];
}

/* The face two cell edges share, or -1. */
static int common_face(int e1, int e2)
{
    int f1[2], f2[2];
    edge_faces(e1, f1);
    edge_faces(e2, f2);
    for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q)
            if (f1[p] == f2[q])
                return f1[p];
    return -1;
}

static int64_t find_key(const uint32_t *keys, int64_t n, uint32_t key)
{
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (keys[mid] == key)
            return mid;
        if (keys[mid] < key)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

int64_t orc_mesh(const int32_t *n, const uint8_t *occ, const uint32_t *keys, int64_t n_keys,
                 uint32_t *tris, int64_t max_tris)
{
    const int64_t nx = n[0], ny = n[1], nz = n[2];
    int64_t T = 0;
    for (int64_t k = 0; k + 1 < nz; ++k)
        for (int64_t j = 0; j + 1 < ny; ++j)
            for (int64_t i = 0; i + 1 < nx; ++i) {
                int inside[8], any = 0, all = 1;
                for (int b = 0; b < 8; ++b) {
                    const int64_t lin = (i + (b & 1)) + nx * ((j + ((b >> 1) & 1)) + ny * (k + ((b >> 2) & 1)));
                    inside[b] = occ[lin] != 0;
                    any |= inside[b];
                    all &= inside[b];
                }
                if (!any || all)
                    continue;
                int next[12], seen[12] = {0};
                cell_segments(inside, next);
                for (int e = 0; e < 12; ++e) {
                    if (next[e] < 0 || seen[e])
                        continue;
                    int loop[12], m = 0;
                    for (int x = e; !seen[x]; x = next[x]) {
                        seen[x] = 1;
                        loop[m++] = x;
                    }
                    /* faces crossed twice by this loop: a segment lies on
                     * the face common to its two edges */
                    int face_segs[6] = {0};
                    for (int q = 0; q < m; ++q) {
                        const int f = common_face(loop[q], loop[(q + 1) % m]);
                        if (f >= 0)
                            ++face_segs[f];
                    }
                    int apex = 0;
                    for (int q = 0; q < m; ++q) {
                        int fa[2];
                        edge_faces(loop[q], fa);
                        if (face_segs[fa[0]] < 2 && face_segs[fa[1]] < 2) {
                            apex = q;
                            break;
                        }
                    }
                    int rot[12];
                    for (int q = 0; q < m; ++q)
                        rot[q] = loop[(apex + q) % m];
                    for (int q = 0; q < m; ++q)
                        loop[q] = rot[q];
                    int64_t idx[12];
                    for (int q = 0; q < m; ++q) {
                        int c0[3], c1[3];
                        cell_edge_ends(loop[q], c0, c1);
                        const int64_t lin = (i + c0[0]) + nx * ((j + c0[1]) + ny * (k + c0[2]));
                        idx[q] = find_key(keys, n_keys, (uint32_t)(3 * lin + loop[q] / 4));
                        if (idx[q] < 0)
                            return -1;
                    }
                    for (int q = 1; q + 1 < m; ++q) {
                        if (T < max_tris) {
                            tris[3 * T + 0] = (uint32_t)idx[0];
                            tris[3 * T + 1] = (uint32_t)idx[q];
                            tris[3 * T + 2] = (uint32_t)idx[q + 1];
                        }
                        ++T;
                    }
                }
            }
    return T;
}
