// Sizes and field offsets of the boundary's structs, printed as JSON, for the
// check that the Python binding's ctypes structures match include/fvv.h.
#include <cstddef>
#include <cstdio>

#include "fvv.h"

#define F(T, f) std::printf("\"%s.%s\": %zu, ", #T, #f, offsetof(T, f))
#define S(T) std::printf("\"%s\": %zu, ", #T, sizeof(T))

int main() {
    std::printf("{");
    S(fvv_camera); F(fvv_camera, P); F(fvv_camera, width); F(fvv_camera, height);
    S(fvv_grid); F(fvv_grid, origin); F(fvv_grid, h); F(fvv_grid, lo); F(fvv_grid, dims);
    S(fvv_roi); F(fvv_roi, lo); F(fvv_roi, hi); F(fvv_roi, count);
    S(fvv_job); F(fvv_job, grid); F(fvv_job, cam_base); F(fvv_job, n_cams); F(fvv_job, width);
    F(fvv_job, height); F(fvv_job, sil_base); F(fvv_job, out_offset);
    S(fvv_limits); F(fvv_limits, max_points); F(fvv_limits, max_jobs);
    S(fvv_tile); F(fvv_tile, persistent_blocks);
    S(fvv_frame_params); F(fvv_frame_params, cams); F(fvv_frame_params, coarse);
    F(fvv_frame_params, hc_um); F(fvv_frame_params, t_np); F(fvv_frame_params, n_steps);
    F(fvv_frame_params, coarse_tile); F(fvv_frame_params, fine_tile);
    F(fvv_frame_params, exit_estimator);
    S(fvv_frame_out); F(fvv_frame_out, d_counts); F(fvv_frame_out, max_rois);
    F(fvv_frame_out, max_fine); F(fvv_frame_out, max_points); F(fvv_frame_out, d_tris);
    F(fvv_frame_out, d_tri_off); F(fvv_frame_out, max_tris);
    S(fvv_soft_camera); F(fvv_soft_camera, R0); F(fvv_soft_camera, t0); F(fvv_soft_camera, omega);
    F(fvv_soft_camera, tau);
    std::printf("\"end\": 0}\n");
    return 0;
}
