// Differentiable soft visual hull on gfx950: a smooth relative of the binary
// hull of Sec. II-B-1 (every camera must see a point inside its silhouette)
// for refining silhouettes and camera poses by gradient descent.
//
//   camera c: X_c = R_c X + t_c, R_c = exp([omega_c]x) R0_c, t_c = t0_c + tau_c;
//             u = fx X_c.x / X_c.z + cx, v = fy X_c.y / X_c.z + cy (pixel (x, y)
//             covers [x, x+1) x [y, y+1), centre at (x + 0.5, y + 0.5));
//   p_c(X)  = bilinear interpolation of sigmoid(L_c) between pixel centres at
//             (u, v), off-image pixels 0, and 0 behind the camera;
//   o(X)    = prod_c p_c(X), loss = sum_v (o_v - target_v)^2.
//
// The adjoint recomputes every sample's projections instead of storing them
// (one lattice at a time), takes d o / d p_c as the product of the other
// cameras' p from prefix and suffix products (no division by a p that may be
// 0), scatters the logit gradient into the four taps, and reduces each
// camera's pose gradient over the lattice: with g = d loss / d X_c,
// d loss / d tau = sum g and d loss / d omega = J_l(omega)^T sum (R X) x g,
// J_l being the left Jacobian of SO(3) (exp([omega + d]x) = exp([J_l d]x)
// exp([omega]x) to first order).
#include <limits.h>
#include <math.h>
#include <string.h>

#include <algorithm>

#include "fvv_internal.h"

namespace fvv {

// ------------------------------------------------------------------ host: rotations
// exp([w]x) = I + a [w]x + b [w]x^2 and J_l(w) = I + b [w]x + c [w]x^2 with
// a = sin t / t, b = (1 - cos t) / t^2, c = (t - sin t) / t^3 (t = |w|), by
// their series below t = 1e-3 (where the closed forms cancel).
void so3_exp_and_left_jacobian(const float w_in[3], double R[9], double J[9]) {
    const double w[3] = {w_in[0], w_in[1], w_in[2]};
    const double t2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2], t = sqrt(t2);
    double a, b, c;
    if (t < 1e-3) {
        a = 1.0 - t2 / 6.0 + t2 * t2 / 120.0;
        b = 0.5 - t2 / 24.0 + t2 * t2 / 720.0;
        c = 1.0 / 6.0 - t2 / 120.0 + t2 * t2 / 5040.0;
    } else {
        a = sin(t) / t;
        b = (1.0 - cos(t)) / t2;
        c = (t - sin(t)) / (t2 * t);
    }
    const double K[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
    double K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k)
                s += K[3 * i + k] * K[3 * k + j];
            K2[3 * i + j] = s;
        }
    for (int i = 0; i < 9; ++i) {
        const double I = (i % 4 == 0) ? 1.0 : 0.0;
        R[i] = I + a * K[i] + b * K2[i];
        J[i] = I + b * K[i] + c * K2[i];
    }
}

bool make_soft_cams(int n, int W, int H, const fvv_soft_camera* in, SoftCamSet* cs,
                    SoftJacobians* jac) {
    memset(cs, 0, sizeof(*cs));
    cs->n = n;
    cs->W = W;
    cs->H = H;
    for (int c = 0; c < n; ++c) {
        const fvv_soft_camera& s = in[c];
        const float* all[5] = {s.K, s.R0, s.t0, s.omega, s.tau};
        const int cnt[5] = {4, 9, 3, 3, 3};
        for (int q = 0; q < 5; ++q)
            for (int k = 0; k < cnt[q]; ++k)
                if (!isfinite(all[q][k]))
                    return false;
        if (!(s.K[0] > 0.0f) || !(s.K[1] > 0.0f))
            return false;
        double E[9], J[9];
        so3_exp_and_left_jacobian(s.omega, E, J);
        SoftCam& d = cs->c[c];
        d.fx = s.K[0];
        d.fy = s.K[1];
        d.cx = s.K[2];
        d.cy = s.K[3];
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) {
                double r = 0;
                for (int k = 0; k < 3; ++k)
                    r += E[3 * i + k] * (double)s.R0[3 * k + j];
                d.R[3 * i + j] = (float)r;
            }
            d.t[i] = (float)((double)s.t0[i] + (double)s.tau[i]);
        }
        for (int i = 0; i < 9; ++i)
            jac->Jl[c][i] = J[i];
    }
    return true;
}

// ------------------------------------------------------------------ device: one camera
struct SoftSample {
    float p;            // bilinear sigmoid value (0 behind the camera)
    float Xc[3];        // camera-space point
    float sg[4];        // sigmoid of taps (x0,y0), (x0+1,y0), (x0,y0+1), (x0+1,y0+1); 0 off-image
    float ax, ay;       // bilinear fractions
    int x0, y0;
    bool front;
};

__device__ __forceinline__ float sigmoidf(float L) { return 1.0f / (1.0f + expf(-L)); }

__device__ __forceinline__ SoftSample soft_sample(const SoftCam& k, const float* __restrict__ L,
                                                  int W, int H, float X, float Y, float Z) {
    SoftSample s;
    s.Xc[0] = __builtin_fmaf(k.R[2], Z, __builtin_fmaf(k.R[1], Y, __builtin_fmaf(k.R[0], X, k.t[0])));
    s.Xc[1] = __builtin_fmaf(k.R[5], Z, __builtin_fmaf(k.R[4], Y, __builtin_fmaf(k.R[3], X, k.t[1])));
    s.Xc[2] = __builtin_fmaf(k.R[8], Z, __builtin_fmaf(k.R[7], Y, __builtin_fmaf(k.R[6], X, k.t[2])));
    s.front = s.Xc[2] > 0.0f;
    const float rz = s.front ? 1.0f / s.Xc[2] : 0.0f;
    // pixel-centre coordinates, clamped where every tap is off-image anyway
    const float su = fminf(fmaxf(k.fx * s.Xc[0] * rz + k.cx - 0.5f, -2.0f), (float)W + 1.0f);
    const float sv = fminf(fmaxf(k.fy * s.Xc[1] * rz + k.cy - 0.5f, -2.0f), (float)H + 1.0f);
    const float fx0 = floorf(su), fy0 = floorf(sv);
    s.ax = su - fx0;
    s.ay = sv - fy0;
    s.x0 = (int)fx0;
    s.y0 = (int)fy0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int x = s.x0 + (q & 1), y = s.y0 + (q >> 1);
        const bool in = s.front && x >= 0 && x < W && y >= 0 && y < H;
        s.sg[q] = in ? sigmoidf(L[(int64_t)y * W + x]) : 0.0f;
    }
    s.p = s.front ? (1.0f - s.ax) * (1.0f - s.ay) * s.sg[0] + s.ax * (1.0f - s.ay) * s.sg[1] +
                        (1.0f - s.ax) * s.ay * s.sg[2] + s.ax * s.ay * s.sg[3]
                  : 0.0f;
    return s;
}

__device__ __forceinline__ void sample_coords(const fvv_grid& g, uint32_t idx, float& X, float& Y,
                                              float& Z) {
    const uint32_t nx = (uint32_t)g.dims[0], ny = (uint32_t)g.dims[1];
    const uint32_t r = idx / nx;
    X = lattice_coord(g.lo[0] + (int)(idx - r * nx), g.h, g.origin[0]);
    Y = lattice_coord(g.lo[1] + (int)(r % ny), g.h, g.origin[1]);
    Z = lattice_coord(g.lo[2] + (int)(r / ny), g.h, g.origin[2]);
}

// Sum over the wave (DPP row shifts and broadcasts; lane 63 holds the total).
__device__ __forceinline__ float wave_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xf, 0xf, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xf, 0xf, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xf, 0xf, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xa, 0xf, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xc, 0xf, false));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), kWave - 1));
}

// ------------------------------------------------------------------ kernels
__global__ __launch_bounds__(kBlock) void soft_zero_kernel(float* __restrict__ f, int64_t nf,
                                                           double* __restrict__ d, int nd) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (int64_t q = i; q < nf; q += (int64_t)gridDim.x * kBlock)
        f[q] = 0.0f;
    if (i < nd)
        d[i] = 0.0;
}

template <bool kLoss>
__global__ __launch_bounds__(kBlock) void soft_fwd_kernel(const SoftCamSet cams, const fvv_grid g,
                                                          const float* __restrict__ logits,
                                                          const float* __restrict__ target,
                                                          float* __restrict__ occ,
                                                          double* __restrict__ loss) {
    __shared__ double s_part[kBlock / kWave];
    const uint32_t V = (uint32_t)((int64_t)g.dims[0] * g.dims[1] * g.dims[2]);
    const int64_t cam_px = (int64_t)cams.W * cams.H;
    double acc = 0.0;
    for (uint32_t idx = blockIdx.x * kBlock + threadIdx.x; idx < V; idx += gridDim.x * kBlock) {
        float X, Y, Z;
        sample_coords(g, idx, X, Y, Z);
        float o = 1.0f;
        for (int c = 0; c < cams.n && o != 0.0f; ++c)
            o *= soft_sample(cams.c[c], logits + c * cam_px, cams.W, cams.H, X, Y, Z).p;
        if (occ)
            occ[idx] = o;
        if (kLoss) {
            const double d = (double)o - (double)target[idx];
            acc += d * d;
        }
    }
    if (kLoss) {
        // block sum in double (wave partials through LDS), one atomic per block
        for (int off = 32; off >= 1; off >>= 1)
            acc += __shfl_xor(acc, off);
        if (lane_id() == 0)
            s_part[threadIdx.x / kWave] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < kBlock / kWave; ++w)
                t += s_part[w];
            unsafeAtomicAdd(loss, t);
        }
    }
}

__device__ __forceinline__ int wave_min_i32(int v) {
    for (int off = kWave / 2; off >= 1; off >>= 1)
        v = min(v, __shfl_xor(v, off));
    return v;
}

__device__ __forceinline__ int wave_max_i32(int v) {
    for (int off = kWave / 2; off >= 1; off >>= 1)
        v = max(v, __shfl_xor(v, off));
    return v;
}

// The adjoint.  A block takes bricks of 8 x 8 x 4 lattice samples, one per
// thread, and walks the cameras in order with the prefix product, the suffix
// products of all cameras' p held in registers (kN: a compile-time bound on the
// camera count).  Per camera, the brick's logit-gradient contributions fall in
// a small pixel window (the brick spans a few pixels): they are summed there
// with LDS atomics and the window is added to the gradient image with one
// global atomic per touched pixel, instead of four contended global atomics
// per sample (all samples along a camera ray hit the same pixels).  Windows
// larger than kWin pixels fall back to global atomics.  A work item is a brick
// and one of kCamGroups camera groups (cameras c = group mod kCamGroups): each
// item forms all cameras' p but does the gradient work of its group only, so
// kCamGroups times as many workgroups share the latency.  acc [n][6]: per camera
// sum of g = d loss / d X_c and of (R X) x g (DPP wave sums, LDS, then double
// atomics per block).
constexpr int kBrickX = 8, kBrickY = 8, kBrickZ = kBlock / (kBrickX * kBrickY);
constexpr int kWin = 4096;
constexpr int kCamGroups = 4;

template <int kN, bool kL2>
__global__ __launch_bounds__(kBlock) void soft_bwd_kernel(const SoftCamSet cams, const fvv_grid g,
                                                          const float* __restrict__ logits,
                                                          const float* __restrict__ target,
                                                          const float* __restrict__ grad_occ,
                                                          const double* __restrict__ scale_p,
                                                          float* __restrict__ grad_logits,
                                                          double* __restrict__ acc) {
    __shared__ float s_acc[kN][6];
    __shared__ float s_win[kWin];
    // window of the item's m-th camera in s_box[m & 1]: min x, min y, max x,
    // max y of the taps (two buffers: a buffer's readers have all passed the
    // next camera's barrier before thread 0 resets it)
    __shared__ int s_box[2][4];
    for (int q = threadIdx.x; q < kN * 6; q += kBlock)
        s_acc[q / 6][q % 6] = 0.0f;
    const int nx = g.dims[0], ny = g.dims[1], nz = g.dims[2];
    const int nbx = (nx + kBrickX - 1) / kBrickX, nby = (ny + kBrickY - 1) / kBrickY;
    const int nbz = (nz + kBrickZ - 1) / kBrickZ;
    const int64_t bricks = (int64_t)nbx * nby * nbz;
    const int64_t cam_px = (int64_t)cams.W * cams.H;
    const float scale = scale_p ? (float)*scale_p : 1.0f;
    const int lx = threadIdx.x % kBrickX, ly = (threadIdx.x / kBrickX) % kBrickY;
    const int lz = threadIdx.x / (kBrickX * kBrickY);
    for (int64_t item = blockIdx.x; item < bricks * kCamGroups; item += gridDim.x) {
        const int64_t br = item / kCamGroups;
        const int group = (int)(item % kCamGroups);
        const int bx = (int)(br % nbx), by = (int)((br / nbx) % nby), bz = (int)(br / nbx / nby);
        const int i = bx * kBrickX + lx, j = by * kBrickY + ly, k = bz * kBrickZ + lz;
        const bool act = i < nx && j < ny && k < nz;
        const uint32_t idx = act ? (uint32_t)(((int64_t)k * ny + j) * nx + i) : 0u;
        float X, Y, Z;
        sample_coords(g, idx, X, Y, Z);
        float p[kN], suf[kN];
#pragma unroll
        for (int c = 0; c < kN; ++c)
            p[c] = c < cams.n ? soft_sample(cams.c[c], logits + c * cam_px, cams.W, cams.H, X, Y, Z).p
                              : 1.0f;
        suf[kN - 1] = 1.0f;
#pragma unroll
        for (int c = kN - 1; c > 0; --c)
            suf[c - 1] = suf[c] * p[c];
        const float o = suf[0] * p[0];
        float go = 0.0f;
        if (act)
            go = (kL2 ? 2.0f * (o - target[idx]) : grad_occ[idx]) * scale;
        float pre = 1.0f;
#pragma unroll
        for (int c = 0; c < kN; ++c) {
            if (c >= cams.n)
                break;
            const float gp = go * pre * suf[c];
            pre *= p[c];
            if (c % kCamGroups != group)
                continue;                      // another work item's camera
            int* const box = s_box[(c / kCamGroups) & 1];
            if (threadIdx.x == 0) {
                box[0] = box[1] = INT_MAX;
                box[2] = box[3] = INT_MIN;
            }
            if (!__syncthreads_or(gp != 0.0f))
                continue;                      // the whole brick has no gradient here
            const SoftCam& cm = cams.c[c];
            const SoftSample sm = soft_sample(cm, logits + c * cam_px, cams.W, cams.H, X, Y, Z);
            const bool live = gp != 0.0f && sm.front;
            // the brick's tap window
            {
                const int a0 = wave_min_i32(live ? sm.x0 : INT_MAX);
                const int a1 = wave_min_i32(live ? sm.y0 : INT_MAX);
                const int a2 = wave_max_i32(live ? sm.x0 + 1 : INT_MIN);
                const int a3 = wave_max_i32(live ? sm.y0 + 1 : INT_MIN);
                if (lane_id() == 0) {
                    atomicMin(&box[0], a0);
                    atomicMin(&box[1], a1);
                    atomicMax(&box[2], a2);
                    atomicMax(&box[3], a3);
                }
            }
            __syncthreads();
            const int wx0 = box[0], wy0 = box[1];
            const int64_t wxn = (int64_t)box[2] - wx0 + 1, wyn = (int64_t)box[3] - wy0 + 1;
            const bool in_lds = box[2] >= wx0 && wxn * wyn <= kWin;   // uniform
            float* gl = grad_logits + c * cam_px;
            const float w4[4] = {(1.0f - sm.ax) * (1.0f - sm.ay), sm.ax * (1.0f - sm.ay),
                                 (1.0f - sm.ax) * sm.ay, sm.ax * sm.ay};
            if (in_lds) {
                for (int q = threadIdx.x; q < (int)(wxn * wyn); q += kBlock)
                    s_win[q] = 0.0f;
                __syncthreads();
            }
            float gx = 0.0f, gy = 0.0f, gz = 0.0f, bxv = 0.0f, byv = 0.0f, bzv = 0.0f;
            if (live) {
                // logits: d p / d L_tap = weight * sigmoid' (taps off-image have sg = 0)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int x = sm.x0 + (q & 1), y = sm.y0 + (q >> 1);
                    if (x >= 0 && x < cams.W && y >= 0 && y < cams.H) {
                        const float v = gp * w4[q] * sm.sg[q] * (1.0f - sm.sg[q]);
                        if (in_lds)
                            atomicAdd(&s_win[(y - wy0) * wxn + (x - wx0)], v);
                        else
                            unsafeAtomicAdd(&gl[(int64_t)y * cams.W + x], v);
                    }
                }
                // pose: d p / d u and d p / d v, then through the projection
                const float du = (1.0f - sm.ay) * (sm.sg[1] - sm.sg[0]) + sm.ay * (sm.sg[3] - sm.sg[2]);
                const float dv = (1.0f - sm.ax) * (sm.sg[2] - sm.sg[0]) + sm.ax * (sm.sg[3] - sm.sg[1]);
                const float rz = 1.0f / sm.Xc[2];
                gx = gp * du * cm.fx * rz;
                gy = gp * dv * cm.fy * rz;
                gz = -(gx * sm.Xc[0] + gy * sm.Xc[1]) * rz;
                // R X = X_c - t
                const float rx = sm.Xc[0] - cm.t[0], ry = sm.Xc[1] - cm.t[1],
                            rzv = sm.Xc[2] - cm.t[2];
                bxv = ry * gz - rzv * gy;
                byv = rzv * gx - rx * gz;
                bzv = rx * gy - ry * gx;
            }
            const float v6[6] = {gx, gy, gz, bxv, byv, bzv};
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const float t = wave_sum(v6[q]);
                if (lane_id() == 0 && t != 0.0f)
                    atomicAdd(&s_acc[c][q], t);
            }
            if (in_lds) {
                __syncthreads();
                for (int q = threadIdx.x; q < (int)(wxn * wyn); q += kBlock) {
                    const float v = s_win[q];
                    if (v != 0.0f)      // only in-image taps were added
                        unsafeAtomicAdd(&gl[(int64_t)(wy0 + q / wxn) * cams.W + (wx0 + q % wxn)], v);
                }
            }
        }
        __syncthreads();   // the next brick's first camera resets a window buffer
    }
    __syncthreads();
    for (int q = threadIdx.x; q < cams.n * 6; q += kBlock)
        if (s_acc[q / 6][q % 6] != 0.0f)
            unsafeAtomicAdd(&acc[q], (double)s_acc[q / 6][q % 6]);
}

// grad_pose[c] = (J_l^T sum (R X) x g, sum g).
__global__ void soft_pose_kernel(const double* __restrict__ acc, const SoftJacobians jac, int n,
                                 double* __restrict__ grad_pose) {
    const int c = threadIdx.x;
    if (c >= n)
        return;
    const double* a = acc + 6 * c;
    const double* J = jac.Jl[c];
    for (int i = 0; i < 3; ++i)
        grad_pose[6 * c + i] = J[i] * a[3] + J[3 + i] * a[4] + J[6 + i] * a[5];
    for (int i = 0; i < 3; ++i)
        grad_pose[6 * c + 3 + i] = a[i];
}

// ------------------------------------------------------------------ launchers
hipError_t launch_soft_forward(fvv_ctx* ctx, const SoftCamSet& cams, const fvv_grid& g,
                               const float* logits, const float* target, float* occ,
                               double* loss, hipStream_t s) {
    const int64_t V = (int64_t)g.dims[0] * g.dims[1] * g.dims[2];
    const unsigned blocks =
        (unsigned)std::min<int64_t>((V + kBlock - 1) / kBlock, (int64_t)ctx->n_cus * 16);
    if (loss) {
        hipLaunchKernelGGL(soft_zero_kernel, dim3(1), dim3(kBlock), 0, s, nullptr, (int64_t)0,
                           loss, 1);
        hipLaunchKernelGGL(soft_fwd_kernel<true>, dim3(blocks), dim3(kBlock), 0, s, cams, g,
                           logits, target, occ, loss);
    } else {
        hipLaunchKernelGGL(soft_fwd_kernel<false>, dim3(blocks), dim3(kBlock), 0, s, cams, g,
                           logits, target, occ, loss);
    }
    return hipGetLastError();
}

hipError_t launch_soft_backward(fvv_ctx* ctx, const SoftCamSet& cams, const SoftJacobians& jac,
                                const fvv_grid& g, const float* logits, const float* target,
                                const float* grad_occ, const double* scale, float* grad_logits,
                                double* grad_pose, hipStream_t s) {
    const int64_t V = (int64_t)g.dims[0] * g.dims[1] * g.dims[2];
    const int64_t npx = (int64_t)cams.n * cams.W * cams.H;
    const unsigned zb = (unsigned)std::min<int64_t>((npx + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(soft_zero_kernel, dim3(zb), dim3(kBlock), 0, s, grad_logits, npx,
                       ctx->d_soft_acc, FVV_MAX_CAMS * 6);
    const int64_t bricks = (int64_t)((g.dims[0] + kBrickX - 1) / kBrickX) *
                           ((g.dims[1] + kBrickY - 1) / kBrickY) *
                           ((g.dims[2] + kBrickZ - 1) / kBrickZ);
    const unsigned blocks =
        (unsigned)std::min<int64_t>(bricks * kCamGroups, (int64_t)ctx->n_cus * 16);
    (void)V;
#define X(KN)                                                                                   \
    if (target)                                                                                 \
        hipLaunchKernelGGL((soft_bwd_kernel<KN, true>), dim3(blocks), dim3(kBlock), 0, s, cams, \
                           g, logits, target, grad_occ, scale, grad_logits, ctx->d_soft_acc);   \
    else                                                                                        \
        hipLaunchKernelGGL((soft_bwd_kernel<KN, false>), dim3(blocks), dim3(kBlock), 0, s,      \
                           cams, g, logits, target, grad_occ, scale, grad_logits,               \
                           ctx->d_soft_acc);
    if (cams.n <= 16) {
        X(16)
    } else {
        X(FVV_MAX_CAMS)
    }
#undef X
    hipLaunchKernelGGL(soft_pose_kernel, dim3(1), dim3(kWave), 0, s, ctx->d_soft_acc, jac, cams.n,
                       grad_pose);
    return hipGetLastError();
}

}  // namespace fvv
