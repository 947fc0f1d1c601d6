/*
 * fvv.h -- C ABI of the MI355X (gfx950) coarse-to-fine visual-hull library.
 *
 * The library implements the reconstruction path of Chen et al., "A Fast
 * Free-viewpoint Video Synthesis Algorithm for Sports Scenes":
 *   1. sparse (coarse) volumetric visual hull over the whole volume  (Sec. II-B-1)
 *   2. 26-adjacency connected components, the size filter of Eq. (1) and the
 *      minimum 3-D bounding box (ROI) of each kept component         (Sec. II-B-2)
 *   3. dense (fine) visual hull inside each ROI only                (Sec. II-B-3)
 *   4. for every grid edge whose endpoints differ, the point where it
 *      leaves the visual hull (the first exit over all cameras, the
 *      minimum of Eq. (3)), which gives the mesh vertices             (Sec. II-C)
 *
 * Conventions shared by every call
 * --------------------------------
 * Camera    P is a row-major 3x4 float32 projection.  A world point (X,Y,Z)
 *           maps to a = P0.X, b = P1.X, w = P2.X, each evaluated as the fused
 *           chain fma(P[4r+2], Z, fma(P[4r+1], Y, fma(P[4r+0], X, P[4r+3]))).
 *           The point is seen by the camera iff w > 0 and pixel
 *           (floor(a/w), floor(b/w)) lies in [0,W) x [0,H), the floors taken of
 *           the exact real quotient; pixel (x, y) covers [x,x+1) x [y,y+1).
 * Silhouette bit-packed uint32 rows, layout [camera][H][wpr], wpr = ceil(W/32);
 *           pixel x of a row is bit (x & 31) of word (x >> 5); pad bits are 0.
 * Grid      a lattice {origin, h, lo, dims}.  Sample (i,j,k), 0 <= i < dims[0]
 *           etc., has global index g = lo + (i,j,k) and world position
 *           fma((float)g_axis, h, origin_axis) on each axis.  Buffers over a
 *           grid are x-fastest: lin = i + dims[0]*(j + dims[1]*k).
 * Occupancy a sample is occupied iff it is seen inside the silhouette of every
 *           camera (Sec. II-B: a voxel falling outside a silhouette is
 *           unoccupied).  Results are bit-exact: they do not depend on launch
 *           shape, tile choice or camera order.
 *
 * Memory: every d_* pointer is device memory owned by the caller; host
 * pointers are read before the call returns.  The library never frees caller
 * memory.  A context owns all scratch, allocated once by fvv_create (all GPU
 * memory is taken at start-up, as the paper's system does), on the device that
 * is current at that time.  Use one context per concurrently used stream.
 *
 * Errors: argument checks run on the host before anything is enqueued and
 * return FVV_EINVAL.  Launch failures return FVV_EDEVICE.  Overflow of an
 * output capacity is detected on the device: the true count is still written,
 * nothing is written past the capacity, and a sticky flag makes the next
 * fvv_check return FVV_ECAPACITY.  Every call except fvv_create, fvv_destroy,
 * fvv_check and the graph helpers is asynchronous on its stream, makes no host
 * synchronisation, and can be captured into a HIP graph.
 */
#ifndef FVV_H
#define FVV_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FVV_MAX_CAMS 32
#define FVV_MAX_STEPS 12

typedef enum {
    FVV_OK = 0,
    FVV_EINVAL = -1,     /* bad argument, rejected before any work is enqueued */
    FVV_ECAPACITY = -2,  /* an output capacity was exceeded (reported by fvv_check) */
    FVV_EDEVICE = -3,    /* a HIP call failed */
    FVV_ENOMEM = -4      /* fvv_create could not allocate its scratch */
} fvv_status;

typedef struct {
    float P[12];          /* row-major 3x4 projection */
    int32_t width, height;
} fvv_camera;

typedef struct {
    float origin[3];      /* world position of global index 0 on each axis */
    float h;              /* lattice spacing (metres) */
    int32_t lo[3];        /* global index of sample (0,0,0) */
    int32_t dims[3];      /* samples per axis, each >= 1 */
} fvv_grid;

typedef struct {
    int32_t lo[3], hi[3]; /* inclusive bounding box, grid-local indices */
    uint32_t count;       /* voxels in the component, N(S) of Eq. (1) */
    uint32_t min_index;   /* smallest linear index in the component */
} fvv_roi;

/* One unit of batched fine carving: a lattice to carve with the cameras
 * cams[cam_base .. cam_base+n_cams) of the camera table, whose silhouettes
 * start at word sil_base of the silhouette buffer (layout [n_cams][height][wpr]),
 * writing dims[0]*dims[1]*dims[2] bytes at byte out_offset of the output. */
typedef struct {
    fvv_grid grid;
    int32_t cam_base, n_cams;
    int32_t width, height;
    int64_t sil_base;
    int64_t out_offset;
} fvv_job;

typedef struct {
    int32_t max_cams;     /* <= FVV_MAX_CAMS */
    int32_t max_w, max_h; /* largest image */
    int64_t max_coarse;   /* largest grid given to fvv_label / fvv_frame (< 2^31) */
    int64_t max_fine;     /* largest total fine samples of one fvv_frame */
    uint32_t max_rois;    /* largest number of ROIs fvv_frame carries to the fine stage */
    uint32_t max_points;  /* largest number of crossing edges of one fvv_frame */
    uint32_t max_jobs;    /* largest job table given to fvv_carve_batched */
} fvv_limits;

/* Tile of the fine/coarse carving kernels: tx*ty threads per workgroup
 * (tx*ty == 256, tx in {16, 32, 64}), each carving tz samples stacked in z. */
typedef struct {
    int32_t tx, ty, tz;
    int32_t persistent_blocks; /* workgroups of the persistent batched launch; 0 = auto */
} fvv_tile;

typedef struct fvv_ctx fvv_ctx;

/* Create a context: allocates all device scratch for the given limits on the
 * current device.  FVV_EINVAL for limits out of range, FVV_ENOMEM if the
 * allocation fails.  *out is NULL on failure. */
fvv_status fvv_create(fvv_ctx **out, const fvv_limits *limits);

/* Free a context's scratch (synchronises the device first).  NULL is a no-op. */
void fvv_destroy(fvv_ctx *ctx);

/* Static text for a status code. */
const char *fvv_status_str(fvv_status s);

/* Wait for `stream`, then report and clear the context's sticky device flags:
 * FVV_EINVAL if a batched carve met a job out of range since the last check,
 * else FVV_ECAPACITY if a capacity was exceeded, else FVV_OK. */
fvv_status fvv_check(fvv_ctx *ctx, hipStream_t stream);

/* Pack n silhouettes, uint8 [n][height][width] (non-zero = foreground, the
 * binary silhouette of Sec. II-A), into d_sils [n][height][wpr].  n >= 1 is
 * not bounded by max_cams (the images of many frames can be packed at once);
 * EINVAL for NULL pointers or a size outside 1..max_w x 1..max_h. */
fvv_status fvv_pack_silhouettes(fvv_ctx *ctx, int32_t n, int32_t width, int32_t height,
                                const uint8_t *d_masks, uint32_t *d_sils, hipStream_t stream);

/* Volumetric visual hull on one lattice (Sec. II-B-1 for the whole volume,
 * Sec. II-B-3 for an ROI): d_occ[lin] = 1 if the sample is occupied, else 0.
 * cams: host array of n_cams (1..max_cams) cameras with identical width and
 * height; d_sils: their silhouettes.  EINVAL on NULL pointers, bad counts,
 * mismatched or oversized images, non-finite P, dims < 1, more than 2^31-1
 * samples, or |global index| >= 2^24. */
fvv_status fvv_carve(fvv_ctx *ctx, int32_t n_cams, const fvv_camera *cams,
                     const uint32_t *d_sils, const fvv_grid *grid, const fvv_tile *tile,
                     uint8_t *d_occ, hipStream_t stream);

/* Connected components and ROIs (Sec. II-B-2).  d_occ (in: occupancy of
 * `grid`, out: occupancy with removed components switched OFF), d_labels
 * (out, int32 per sample): components are maximal sets of ON samples linked by
 * 26-adjacency; a component S is kept iff t_np <= N(S) <= t_nb (Eq. (1), read
 * as the sentence after it states); kept components are numbered 1..K in
 * ascending order of their smallest linear index, labels are 0 elsewhere.
 * d_rois[t-1] (t <= max_rois) receives component t's box; *d_n_rois receives
 * K (device).  K > max_rois sets the ECAPACITY flag.  EINVAL if the grid
 * exceeds max_coarse, pointers are NULL or t_np > t_nb. */
fvv_status fvv_label(fvv_ctx *ctx, const fvv_grid *grid, uint8_t *d_occ, int32_t *d_labels,
                     uint32_t t_np, uint32_t t_nb, fvv_roi *d_rois, uint32_t max_rois,
                     uint32_t *d_n_rois, hipStream_t stream);

/* Fine lattice of each ROI (Sec. II-B-3: each ROI is carved as its own
 * volume).  Host-only, pure integer arithmetic.  Lattices share the coarse
 * origin; spacings are integer micrometres hc_um (coarse) and hf_um (fine)
 * and the fine spacing is h = (float)((double)hf_um * 1e-6).  Per axis, with
 * A = coarse.lo + roi.lo and B = coarse.lo + roi.hi (global coarse indices):
 * fine indices [floor((A-1) hc/hf), ceil((B+1) hc/hf)], clamped to the fine
 * samples inside the coarse lattice's extent, i.e. the box dilated by one
 * coarse cell.  EINVAL on NULL pointers or non-positive spacings. */
fvv_status fvv_roi_grids(const fvv_grid *coarse, int64_t hc_um, int64_t hf_um,
                         const fvv_roi *rois, uint32_t n, fvv_grid *out);

/* Exit points of one carved ROI (Sec. II-C).  d_occ_fine: occupancy of `roi`.
 * Every lattice edge (p, p+e_axis) with both ends in the grid and
 * occ(p) != occ(p+e_axis) is a crossing edge with key 3*lin(p)+axis; keys are
 * written to d_keys in ascending order.  For each, n_steps (1..12) bisection
 * steps on the edge parameter t (0 at the ON end, 1 at the OFF end) test the
 * midpoint with the occupancy test above; the vertex is the final bracket's
 * midpoint t* = (lo+hi)/2, d_xyz[3e..3e+2] its world position (axis
 * coordinate fma(g_on + d*t*, h, origin), d = +1 or -1 toward the OFF end).
 * *d_n_points receives the edge count E; E > max_points sets ECAPACITY and
 * only the first max_points are written.  EINVAL as fvv_carve, plus n_steps
 * out of range or |global index| >= 2^(23 - n_steps). */
fvv_status fvv_surface(fvv_ctx *ctx, const fvv_grid *roi, const uint8_t *d_occ_fine,
                       int32_t n_cams, const fvv_camera *cams, const uint32_t *d_sils,
                       int32_t n_steps, uint32_t *d_keys, float *d_xyz, uint32_t max_points,
                       uint32_t *d_n_points, hipStream_t stream);

/* Allocation-free variant of fvv_surface, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, results and kernels as fvv_surface,
 * without a context.  Its scratch (the lattice's job table, crossing edges per
 * work item, fine bitmap, and the silhouettes in 8 x 8-pixel blocks when
 * n_cams * ceil(W / 8) * ceil(H / 8) <= FVV_NOALLOC_TILE_WORDS; larger rigs
 * take a slower path of the same kernels) is one static device array of about
 * 16 MiB on each GPU the library runs on, held until the process ends; the
 * call allocates no device memory and calls no allocating library routine.
 * Limits: the
 * lattice's fine bitmap, ny * nz * ceil(nx / 64) words, at most
 * FVV_NOALLOC_BITMAP_WORDS (else EINVAL); at most FVV_MAX_CAMS cameras of up
 * to 65536 x 65536 pixels.  Capacity: *d_n_points always receives the edge
 * count E, and only the first max_points edges are written when E exceeds it;
 * with no context there is no sticky ECAPACITY, so compare *d_n_points with
 * max_points.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (several streams or threads) race and must be serialised
 * by the caller.  EDEVICE when the array's device address cannot be looked up
 * or a launch fails. */
#define FVV_NOALLOC_BITMAP_WORDS (1 << 20)
#define FVV_NOALLOC_TILE_WORDS (1 << 20)
fvv_status fvv_surface_noalloc(const fvv_grid *roi, const uint8_t *d_occ_fine, int32_t n_cams,
                               const fvv_camera *cams, const uint32_t *d_sils, int32_t n_steps,
                               uint32_t *d_keys, float *d_xyz, uint32_t max_points,
                               uint32_t *d_n_points, hipStream_t stream);

/* Batched fine carving (Sec. II-B-3 over many ROIs, of one or many frames) in
 * ONE persistent launch.  d_jobs: n_jobs jobs (device, <= max_jobs); d_cams:
 * device camera table; output bytes as each job states.  The output is
 * byte-identical to carving each job with fvv_carve, whatever the tile.
 * With tile->tz == 4 (and for tile == NULL, the default 64x4x4 tile) the
 * cameras are culled per 4x4x4 box of samples (a camera whose padded pixel
 * rectangle over the box holds no foreground rejects the box; one whose
 * rectangle is all foreground accepts it) and the tiles are split statically
 * over the XCDs; other depths test every sample against every camera, the
 * workgroups taking tiles from a device counter.  A job with n_cams outside
 * 1..FVV_MAX_CAMS, an image side outside 1..65536, an empty lattice or a
 * negative base or offset is skipped, and the next fvv_check reports
 * FVV_EINVAL.  Calls on one context must not overlap (they share its
 * scratch). */
fvv_status fvv_carve_batched(fvv_ctx *ctx, const fvv_job *d_jobs, uint32_t n_jobs,
                             const fvv_camera *d_cams, const uint32_t *d_sils,
                             uint8_t *d_occ_out, const fvv_tile *tile, hipStream_t stream);

/* Tile selection for fvv_carve_batched (the autotuner's measurement): for
 * each of the n_cands candidate tiles, one untimed call and then `reps`
 * (1..1000) calls between two HIP events on `stream`; ms[i] receives the
 * mean milliseconds per call of candidate i, *best the index of the fastest.
 * Every call writes the same bytes to d_occ_out.  Synchronous.  EINVAL for
 * an invalid candidate or argument (nothing is run then), else the status of
 * the first failing call. */
fvv_status fvv_tune_carve_batched(fvv_ctx *ctx, const fvv_job *d_jobs, uint32_t n_jobs,
                                  const fvv_camera *d_cams, const uint32_t *d_sils,
                                  uint8_t *d_occ_out, const fvv_tile *cands, uint32_t n_cands,
                                  int32_t reps, float *ms, uint32_t *best, hipStream_t stream);

/* ---------------------------------------------------------------- one frame
 * The whole path for one frame with every intermediate on the device, so it
 * can run as a single HIP graph: carve the coarse grid, label it, turn each
 * kept ROI into a fine job (fvv_roi_grids' arithmetic, on the device), carve
 * all ROIs in one persistent launch, and find the exit points of every ROI's
 * crossing edges.  Outputs (device, caller-owned):
 *   d_occ_coarse  [coarse samples]       filtered coarse occupancy
 *   d_labels      [coarse samples]       component labels
 *   d_rois        [max_rois]             ROI boxes; counts[0] = K
 *   d_jobs        [max_rois]             fine lattice of each ROI (as fvv_job)
 *   d_occ_fine    [max_fine]             fine occupancy, ROI t at d_jobs[t].out_offset
 *   d_keys/d_xyz  [max_points]           crossing edges of all ROIs, ROI-major
 *   d_point_off   [max_rois + 1]         first edge of each ROI
 *   d_counts      [4]                    K, fine samples, edges, ROIs carried
 * ROIs whose fine lattices do not fit max_fine are not carried (ECAPACITY). */
typedef struct {
    int32_t n_cams;
    fvv_camera cams[FVV_MAX_CAMS];
    fvv_grid coarse;
    int64_t hc_um, hf_um;
    uint32_t t_np, t_nb;
    int32_t n_steps;
    fvv_tile coarse_tile, fine_tile;
    /* how the exit points are found: FVV_EXIT_BISECTION (n_steps bisection
     * steps against the occupancy test, as fvv_surface) or FVV_EXIT_BRESENHAM
     * (the paper's image-space isovalue, as fvv_isovalue) */
    int32_t exit_estimator;
} fvv_frame_params;
#define FVV_EXIT_BISECTION 0
#define FVV_EXIT_BRESENHAM 1

typedef struct {
    uint8_t *d_occ_coarse;
    int32_t *d_labels;
    fvv_roi *d_rois;
    fvv_job *d_jobs;
    uint8_t *d_occ_fine;
    uint32_t *d_keys;
    float *d_xyz;
    uint32_t *d_point_off;
    uint32_t *d_counts;
    uint32_t max_rois;
    int64_t max_fine;
    uint32_t max_points;
    /* optional marching-cubes triangles of every ROI (as fvv_mesh, vertex
     * indices into d_keys / d_xyz of the frame): NULL d_tris for none.
     * d_tri_off: [max_rois + 1], the ROI's first triangle, [K] the total
     * (clamped to 2^32 - 1, ECAPACITY past max_tris). */
    uint32_t *d_tris;
    uint32_t *d_tri_off;
    uint32_t max_tris;
} fvv_frame_out;

/* Enqueue the whole frame on `stream`.  d_masks: the frame's uint8
 * silhouettes [n_cams][H][W], packed into d_sils first; or NULL when d_sils
 * already holds the packed silhouettes.  events: NULL, or FVV_FRAME_EVENTS
 * HIP events: the first FVV_FRAME_STAGE_EVENTS are recorded on `stream` at
 * the start and after each stage (pack, coarse carve, labelling, fine jobs +
 * fine carve, crossing edges, exit points) -- a per-stage timing of the
 * frame; the last four take the start and end times of the fine-carve kernel
 * and of the exit-point kernel themselves (hipExtLaunchKernel), so their
 * differences are the two kernels' execution times.  Events must be NULL
 * while the stream is captured into a graph.  EINVAL as the individual calls,
 * and for spacings hc_um or hf_um above 2^28.  Calls on one context must not
 * overlap (they share its scratch). */
#define FVV_FRAME_STAGE_EVENTS 7
#define FVV_FRAME_EVENTS 11
fvv_status fvv_frame(fvv_ctx *ctx, const fvv_frame_params *params, const uint8_t *d_masks,
                     uint32_t *d_sils, const fvv_frame_out *out, hipEvent_t *events,
                     hipStream_t stream);

/* Triangles of the isosurface over the cells of one lattice (Sec. II-C: with
 * a vertex on every crossing edge, the surface follows the marching-cubes
 * configurations, expressed as triangles).  A cell's surface crosses exactly
 * its edges whose two samples differ, one vertex per crossing edge.  The
 * configurations (the paper gives no table) follow a face rule: on each cell
 * face the crossing edges are joined by segments (with two diagonal occupied
 * corners each is cut off alone), oriented with the face's occupied part on
 * their right seen from outside the cell; the segments chain into loops, each
 * cut into a fan of triangles (v0, v_i, v_i+1) from the first vertex, in loop
 * order from its smallest cell edge, that lies on no face the loop crosses
 * twice.  Triangles face away from the occupied side and the surface is
 * closed wherever it does not reach the lattice's border.  Cell corners are
 * b = dx + 2 dy + 4 dz, cell edges 4 a + u + 2 v (axis a; u, v the corner
 * coordinates on the other two axes in increasing order).
 *   d_occ:    occupancy of `grid` (device, x fastest), as for fvv_surface;
 *   d_keys:   its crossing edges, ascending (fvv_surface's output), the first
 *             min(*d_n_keys, max_keys) of them valid (*d_n_keys device);
 *   d_tris:   out, uint32 [max_tris][3]: indices into d_keys (so into the
 *             exit points), by cell in linear order (x fastest), loops by
 *             their smallest cell edge;
 *   d_n_tris: out (device), the triangle count.
 * More than max_tris triangles (the first max_tris are written, the count is
 * complete), or a crossing edge missing from the keys (truncated keys, or keys
 * that are not this occupancy's crossing edges), set the ECAPACITY flag; a
 * missing vertex is written as 0xffffffff.  EINVAL on NULL pointers, zero
 * capacities, empty dims, or a lattice beyond 0x55555555 samples or whose fine
 * bitmap exceeds the context's (as for fvv_surface).  Uses the context's
 * scratch: calls on one context must not overlap. */
fvv_status fvv_mesh(fvv_ctx *ctx, const fvv_grid *grid, const uint8_t *d_occ,
                    const uint32_t *d_keys, const uint32_t *d_n_keys, uint32_t max_keys,
                    uint32_t *d_tris, uint32_t max_tris, uint32_t *d_n_tris, hipStream_t stream);

/* The paper's own isovalue of crossing edges (Sec. II-C, Eq. (2)-(3)), for
 * comparison with the exit points of fvv_surface (which bisect the 3-D edge
 * parameter against the occupancy test).  In camera i the edge's two samples
 * project to pixels P_on (the occupied sample's) and P_off -- the exact floor
 * of each fp32 projection (the occupancy test's), P_off clamped to
 * [-8, dim + 8] -- and the line of pixels from P_on to P_off is traced with
 * Bresenham's integer algorithm (all octants: error term dx - dy, a step
 * along x when twice the error is at least -dy, along y when it is at most
 * dx).  P_i is the last pixel before the first one that is background or off
 * the image; lambda_i = |P_i - P_on| / |P_off - P_on| (Eq. (2)), 1 when the
 * line is foreground to its end, 0 when P_on is not foreground or either
 * sample is behind the camera.  lambda = min over cameras (Eq. (3)), taken on
 * lambda_i^2 as the IEEE double quotient of the integer squared lengths, then
 * rounded to float from its square root.
 *   d_occ, cams, d_sils: the lattice's occupancy and the cameras, as for
 *             fvv_surface (n_cams at most the context's max_cams);
 *   d_keys:   crossing edges 3*lin+axis of `grid` (fvv_surface's output), the
 *             first min(*d_n_keys, max_keys) of them used (*d_n_keys device);
 *   d_lambda: out, float [max_keys]: lambda per key (NaN for a key that names
 *             no edge of the lattice);
 *   d_xyz:    out (or NULL), float [max_keys][3]: the point at lambda along
 *             the edge from its occupied sample, the axis coordinate as
 *             fmaf(g_on + d*lambda, h, origin) (d = +-1 toward the other
 *             sample), the other two the lattice values.
 * EINVAL on NULL pointers, zero max_keys, an invalid grid or camera set, or a
 * lattice beyond 0x55555555 samples.  No context scratch is used. */
fvv_status fvv_isovalue(fvv_ctx *ctx, const fvv_grid *grid, const uint8_t *d_occ, int32_t n_cams,
                        const fvv_camera *cams, const uint32_t *d_sils, const uint32_t *d_keys,
                        const uint32_t *d_n_keys, uint32_t max_keys, float *d_lambda,
                        float *d_xyz, hipStream_t stream);

/* Depth images and visibility of a triangle mesh (Sec. II-D, Eq. (4)) in
 * every camera.  Readings of what the paper leaves open:
 *   - a triangle's distance is the camera-plane distance (the projection's
 *     third row, w) of its centroid ((v0 + v1) + v2) / 3 (fp32);
 *   - it covers pixel (x, y) when the pixel centre (x + 0.5, y + 0.5) lies on
 *     the same side of the three edges of the projected triangle (vertices
 *     (a/w, b/w), IEEE fp32 division): the edge functions
 *     (x1 - x0)(py - y0) - (y1 - y0)(px - x0), in fp32 in that order, all
 *     >= 0 or all <= 0.  Triangles with a vertex at w <= 0, of zero area (the
 *     first edge's function at the third vertex is 0), with a non-positive
 *     centroid distance, or naming a vertex at or past the vertex count (the
 *     mesh's 0xffffffff) cover nothing;
 *   - Eq. (4): a pixel's depth is the minimum distance of the triangles
 *     covering it, +inf where none does;
 *   - a triangle is visible in camera c when its centroid's distance is
 *     positive, the centroid projects into pixel (floor(a/w), floor(b/w))
 *     inside the image, and distance - depth there <= t_v (fp32).
 *   d_xyz:   vertices, float [max_vertices][3] (e.g. the exit points), the
 *            first min(*d_n_vertices, max_vertices) valid (*d_n_vertices
 *            device);
 *   d_tris:  uint32 [max_tris][3] vertex indices (fvv_mesh's output), the
 *            first min(*d_n_tris, max_tris) used;
 *   d_depth: out, float [n_cams][H][W], every pixel written;
 *   d_vis:   out, uint32 [max_tris]: bit c set when the triangle is visible in
 *            camera c (the first min(*d_n_tris, max_tris) written).
 * EINVAL on NULL pointers, zero capacities, an invalid camera set or a
 * non-finite t_v.  No context scratch is used. */
fvv_status fvv_visibility(fvv_ctx *ctx, int32_t n_cams, const fvv_camera *cams,
                          const float *d_xyz, const uint32_t *d_n_vertices, uint32_t max_vertices,
                          const uint32_t *d_tris, const uint32_t *d_n_tris, uint32_t max_tris,
                          float t_v, float *d_depth, uint32_t *d_vis, hipStream_t stream);

/* A measurement aid, not part of the path: the rate at which the GPU serves
 * 4-byte words from the device table d_table (n_words >= 64 words, e.g. a
 * frame's packed silhouettes), read coalesced within each wave (64
 * consecutive words) at pseudo-random wave offsets -- the gather ceiling of
 * the carve.  One untimed launch, then `reps` launches between HIP events on
 * `stream`; the call waits for them on the host and *words_per_s receives the
 * words read per second.  d_table is only read (caller-owned); d_sink: device
 * scratch of at least 16384 * 256 uint32, caller-owned, overwritten with lane
 * sums.  EINVAL on NULL pointers, n_words < 64 or reps outside [1, 1000];
 * EDEVICE on a HIP error. */
fvv_status fvv_gather_peak(fvv_ctx *ctx, const uint32_t *d_table, uint32_t n_words,
                           uint32_t *d_sink, int32_t reps, double *words_per_s,
                           hipStream_t stream);

/* ---------------------------------------------------------------- soft hull
 * A differentiable relative of the binary hull of Sec. II-B-1 (not in the
 * paper), for refining silhouette logits and camera poses by gradient descent.
 * Camera c maps a world point X to X_c = R X + t with R = exp([omega]x) R0 and
 * t = t0 + tau (a 6-DoF perturbation of the calibrated pose), and to the
 * continuous pixel position u = fx X_c.x / X_c.z + cx, v = fy X_c.y / X_c.z + cy
 * (pixel (x, y) covers [x, x+1) x [y, y+1), its centre is (x + 0.5, y + 0.5)).
 * p_c(X) is the bilinear interpolation of sigmoid(logits_c) between pixel
 * centres at (u, v), off-image pixels counting 0, and 0 behind the camera; the
 * soft occupancy of a lattice sample is o = prod_c p_c, and the L2 loss
 * against a target occupancy is sum_v (o_v - target_v)^2.  fp32 arithmetic. */
typedef struct {
    float K[4];      /* fx, fy, cx, cy (pixels) */
    float R0[9];     /* calibrated world->camera rotation, row-major */
    float t0[3];     /* calibrated translation: X_cam = R0 X + t0 */
    float omega[3];  /* rotation perturbation (radians), R = exp([omega]x) R0 */
    float tau[3];    /* translation perturbation (metres), t = t0 + tau */
} fvv_soft_camera;

/* Soft occupancy of `grid` (device output d_occ [samples], x fastest; may be
 * NULL) and, with d_target (device [samples]) given, the loss into *d_loss
 * (device double; overwritten).  cams: host array of n_cams (1..max_cams)
 * cameras; d_logits: device float [n_cams][height][width].  EINVAL on NULL
 * logits or cameras, no output, d_loss without d_target, bad counts or sizes,
 * non-finite camera values, non-positive focal lengths, or a grid as for
 * fvv_carve. */
fvv_status fvv_soft_forward(fvv_ctx *ctx, const fvv_grid *grid, int32_t n_cams,
                            const fvv_soft_camera *cams, int32_t width, int32_t height,
                            const float *d_logits, const float *d_target, float *d_occ,
                            double *d_loss, hipStream_t stream);

/* Adjoint of fvv_soft_forward, recomputing every sample (nothing is stored
 * between the calls).  The upstream gradient per sample is
 * scale * 2 (o - target) with d_target (the L2 loss), else scale * d_grad_occ
 * (device float [samples]); exactly one of the two is given.  scale:
 * device double scalar, or NULL for 1.  Outputs (device, overwritten):
 * d_grad_logits float [n_cams][height][width]; d_grad_pose double [n_cams][6],
 * the derivatives with respect to omega (3) then tau (3).  Float atomics
 * order the sums, so results vary in the last bits between runs.  EINVAL as
 * the forward, plus missing outputs or both or neither upstream input.
 * Calls on one context must not overlap (they share its pose accumulators). */
fvv_status fvv_soft_backward(fvv_ctx *ctx, const fvv_grid *grid, int32_t n_cams,
                             const fvv_soft_camera *cams, int32_t width, int32_t height,
                             const float *d_logits, const float *d_target,
                             const float *d_grad_occ, const double *d_scale,
                             float *d_grad_logits, double *d_grad_pose, hipStream_t stream);

/* Capture fvv_frame (with fixed arguments, no events) into an executable HIP
 * graph.  The capture runs on an internal stream; the graph replays the frame
 * with the same pointers.  Release with fvv_graph_destroy. */
typedef struct fvv_graph fvv_graph;
fvv_status fvv_frame_graph_create(fvv_ctx *ctx, const fvv_frame_params *params,
                                  const uint8_t *d_masks, uint32_t *d_sils,
                                  const fvv_frame_out *out, fvv_graph **graph);
/* fvv_carve_batched captured as a HIP graph with the same arguments (the job
 * table, cameras and silhouettes are read when the graph runs). */
fvv_status fvv_carve_batched_graph_create(fvv_ctx *ctx, const fvv_job *d_jobs, uint32_t n_jobs,
                                          const fvv_camera *d_cams, const uint32_t *d_sils,
                                          uint8_t *d_occ_out, const fvv_tile *tile,
                                          fvv_graph **graph);
fvv_status fvv_graph_launch(fvv_graph *graph, hipStream_t stream);
void fvv_graph_destroy(fvv_graph *graph);

#ifdef __cplusplus
}
#endif
#endif /* FVV_H */
