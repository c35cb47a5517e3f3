// Training loss of eq. `loss` without its perceptual term,
//     L = (1 - lam) mean |x - y| + lam (1 - mean SSIM(x, y)),
// and dL/dx, for planar [C][H][W] binary32 images (lam = lambda_1 = 0.2 in
// the paper's experimental settings).  SSIM per channel from an 11 x 11
// Gaussian window (sigma 1.5, weights summing to 1), the image zero outside
// its borders, c1 = 0.01^2, c2 = 0.03^2.
//
// Two passes over 64 x 16 output tiles, each tile staged in LDS with a
// 5-pixel halo and blurred as one pass along rows and one along columns:
//   k_ssim_fwd  window statistics of x and y -> the SSIM map; per-tile sums
//               of SSIM and |x - y| (binary64) and, when a gradient is
//               wanted, the three per-pixel coefficients of dL/dx:
//               dL/d mu_x, dL/d E[x^2], dL/d E[xy];
//   k_ssim_bwd  dL/dx = blur(dL/d mu_x) + 2 x blur(dL/d E[x^2])
//               + y blur(dL/d E[xy]) + (1 - lam)/n sign(x - y)
//               (the window is symmetric, so the adjoint of the zero-filled
//               blur is the same blur);
//   k_loss_sum  the tile sums in a fixed order -> L (binary64, stored as
//               binary32): the result does not depend on scheduling.
// Everything is HBM-bound: x and y are read twice, three coefficient planes
// written and read once, the gradient written once.
#include <math.h>

#include <string>

#include "ctx.h"

using namespace dgs;

namespace {

constexpr int kTaps = 11, kRad = 5;
constexpr int kTileW = 64, kTileH = 16;
constexpr int kRows = kTileH + 2 * kRad;  // staged rows
constexpr int kCols = kTileW + 2 * kRad;  // staged columns
constexpr int kThreads = 256;             // 64 columns x 4 row groups
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

struct Window {
    float g[kTaps];
};

struct LossArgs {
    const float* x;
    const float* y;
    int C, H, W;
    float lam;
    float dls;       // dL/dSSIM at every pixel: -lam / n
    float l1c;       // (1 - lam) / n
    float* coef;     // [3][C][H][W], null: loss only
    double* part;    // [tiles][2]: sum of SSIM, sum of |x - y|
    float* grad;     // [C][H][W]
};

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ __launch_bounds__(kThreads) void k_ssim_fwd(LossArgs a, Window w) {
    __shared__ float sx[kRows][kCols + 1], sy[kRows][kCols + 1];
    __shared__ float hs[5][kRows][kTileW];  // row sums of x, y, x^2, y^2, xy
    __shared__ double red[2][kThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, grp = tid >> 6;
    const int c = blockIdx.z, ty0 = blockIdx.y * kTileH, tx0 = blockIdx.x * kTileW;
    const size_t plane = (size_t)a.H * a.W;
    const float* X = a.x + c * plane;
    const float* Y = a.y + c * plane;
    for (int i = tid; i < kRows * kCols; i += kThreads) {
        const int r = i / kCols, q = i - r * kCols;
        const int gy = ty0 - kRad + r, gx = tx0 - kRad + q;
        const bool in = gy >= 0 && gy < a.H && gx >= 0 && gx < a.W;
        sx[r][q] = in ? X[(size_t)gy * a.W + gx] : 0.0f;
        sy[r][q] = in ? Y[(size_t)gy * a.W + gx] : 0.0f;
    }
    __syncthreads();
    for (int r = grp; r < kRows; r += kThreads / 64) {
        float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f, s4 = 0.0f;
#pragma unroll
        for (int i = 0; i < kTaps; i++) {
            const float xv = sx[r][lane + i], yv = sy[r][lane + i], g = w.g[i];
            s0 = fmaf(g, xv, s0);
            s1 = fmaf(g, yv, s1);
            s2 = fmaf(g, xv * xv, s2);
            s3 = fmaf(g, yv * yv, s3);
            s4 = fmaf(g, xv * yv, s4);
        }
        hs[0][r][lane] = s0;
        hs[1][r][lane] = s1;
        hs[2][r][lane] = s2;
        hs[3][r][lane] = s3;
        hs[4][r][lane] = s4;
    }
    __syncthreads();
    const int gx = tx0 + lane;
    double ssum = 0.0, l1sum = 0.0;
#pragma unroll
    for (int k = 0; k < kTileH / 4; k++) {
        const int ro = grp * (kTileH / 4) + k, gy = ty0 + ro;
        if (gy >= a.H || gx >= a.W) continue;
        float m[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int i = 0; i < kTaps; i++) {
            const float g = w.g[i];
#pragma unroll
            for (int t = 0; t < 5; t++) m[t] = fmaf(g, hs[t][ro + i][lane], m[t]);
        }
        const float mx = m[0], my = m[1];
        const float sxx = m[2] - mx * mx, syy = m[3] - my * my, sxy = m[4] - mx * my;
        const float a1 = 2.0f * mx * my + kC1, a2 = 2.0f * sxy + kC2;
        const float b1 = mx * mx + my * my + kC1, b2 = sxx + syy + kC2;
        const float s = (a1 * a2) / (b1 * b2);
        const float xv = sx[ro + kRad][lane + kRad], yv = sy[ro + kRad][lane + kRad];
        ssum += (double)s;
        l1sum += (double)fabsf(xv - yv);
        if (a.coef) {
            // S = a1 a2 / (b1 b2): d/d mu_x through a1 (2 mu_y), a2 (-2 mu_y),
            // b1 (2 mu_x), b2 (-2 mu_x); d/d E[x^2] through b2; d/d E[xy] through a2
            const float ds = a.dls * s;
            const size_t p = c * plane + (size_t)gy * a.W + gx, n = (size_t)a.C * plane;
            a.coef[p] = ds * (2.0f * my / a1 - 2.0f * my / a2 - 2.0f * mx / b1 + 2.0f * mx / b2);
            a.coef[n + p] = -ds / b2;
            a.coef[2 * n + p] = 2.0f * ds / a2;
        }
    }
    ssum = wave_sum(ssum);
    l1sum = wave_sum(l1sum);
    if (lane == 0) {
        red[0][grp] = ssum;
        red[1][grp] = l1sum;
    }
    __syncthreads();
    if (tid == 0) {
        const size_t t = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        double s = 0.0, l = 0.0;
        for (int i = 0; i < kThreads / 64; i++) {
            s += red[0][i];
            l += red[1][i];
        }
        a.part[2 * t] = s;
        a.part[2 * t + 1] = l;
    }
}

__global__ __launch_bounds__(kThreads) void k_ssim_bwd(LossArgs a, Window w) {
    __shared__ float sc[3][kRows][kCols + 1];
    __shared__ float hs[3][kRows][kTileW];
    const int tid = threadIdx.x, lane = tid & 63, grp = tid >> 6;
    const int c = blockIdx.z, ty0 = blockIdx.y * kTileH, tx0 = blockIdx.x * kTileW;
    const size_t plane = (size_t)a.H * a.W, n = (size_t)a.C * plane;
    const float* cf = a.coef + c * plane;
    for (int i = tid; i < kRows * kCols; i += kThreads) {
        const int r = i / kCols, q = i - r * kCols;
        const int gy = ty0 - kRad + r, gx = tx0 - kRad + q;
        const bool in = gy >= 0 && gy < a.H && gx >= 0 && gx < a.W;
        const size_t p = (size_t)gy * a.W + gx;
        sc[0][r][q] = in ? cf[p] : 0.0f;
        sc[1][r][q] = in ? cf[n + p] : 0.0f;
        sc[2][r][q] = in ? cf[2 * n + p] : 0.0f;
    }
    __syncthreads();
    for (int r = grp; r < kRows; r += kThreads / 64) {
        float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
#pragma unroll
        for (int i = 0; i < kTaps; i++) {
            const float g = w.g[i];
            s0 = fmaf(g, sc[0][r][lane + i], s0);
            s1 = fmaf(g, sc[1][r][lane + i], s1);
            s2 = fmaf(g, sc[2][r][lane + i], s2);
        }
        hs[0][r][lane] = s0;
        hs[1][r][lane] = s1;
        hs[2][r][lane] = s2;
    }
    __syncthreads();
    const int gx = tx0 + lane;
#pragma unroll
    for (int k = 0; k < kTileH / 4; k++) {
        const int ro = grp * (kTileH / 4) + k, gy = ty0 + ro;
        if (gy >= a.H || gx >= a.W) continue;
        float b0 = 0.0f, b1 = 0.0f, b2 = 0.0f;
#pragma unroll
        for (int i = 0; i < kTaps; i++) {
            const float g = w.g[i];
            b0 = fmaf(g, hs[0][ro + i][lane], b0);
            b1 = fmaf(g, hs[1][ro + i][lane], b1);
            b2 = fmaf(g, hs[2][ro + i][lane], b2);
        }
        const size_t p = c * plane + (size_t)gy * a.W + gx;
        const float xv = a.x[p], yv = a.y[p];
        const float sg = (float)(xv > yv) - (float)(xv < yv);
        a.grad[p] = fmaf(a.l1c, sg, fmaf(yv, b2, fmaf(2.0f * xv, b1, b0)));
    }
}

// One workgroup: the tile sums in a fixed order, then L.
__global__ __launch_bounds__(kThreads) void k_loss_sum(const double* part, size_t tiles, double n, double lam,
                                                       float* loss) {
    __shared__ double red[2][kThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, grp = tid >> 6;
    double s = 0.0, l = 0.0;
    for (size_t t = tid; t < tiles; t += kThreads) {
        s += part[2 * t];
        l += part[2 * t + 1];
    }
    s = wave_sum(s);
    l = wave_sum(l);
    if (lane == 0) {
        red[0][grp] = s;
        red[1][grp] = l;
    }
    __syncthreads();
    if (tid == 0) {
        double ss = 0.0, ll = 0.0;
        for (int i = 0; i < kThreads / 64; i++) {
            ss += red[0][i];
            ll += red[1][i];
        }
        *loss = (float)((1.0 - lam) * ll / n + lam * (1.0 - ss / n));
    }
}

// The 11 window weights: exp(-t^2 / (2 sigma^2)) for t = -5..5, divided by
// their sum (binary64, then rounded).
Window make_window() {
    double g[kTaps], sum = 0.0;
    for (int i = 0; i < kTaps; i++) {
        const double t = (double)(i - kRad) / 1.5;
        g[i] = exp(-0.5 * t * t);
        sum += g[i];
    }
    Window w;
    for (int i = 0; i < kTaps; i++) w.g[i] = (float)(g[i] / sum);
    return w;
}

template <class T>
hipError_t ensure_buf(T*& p, int64_t& cap, int64_t want, hipStream_t st) {
    if (want <= cap && p) return hipSuccess;
    if (p) {
        hipStreamSynchronize(st);
        hipFree(p);
        p = nullptr;
        cap = 0;
    }
    const hipError_t e = hipMalloc((void**)&p, sizeof(T) * (size_t)want);
    if (e == hipSuccess) cap = want;
    return e;
}

}  // namespace

extern "C" {

dgs_status dgs_loss_l1_ssim(dgs_ctx c, const float* image, const float* target, int32_t channels, int32_t height,
                            int32_t width, float lambda, float* loss, float* grad_image) {
    if (!c) return DGS_ERR_INVALID_ARG;
    if (channels < 1 || channels > 65535 || height < 1 || height > 32767 || width < 1 || width > 32767) {
        c->err = "loss: channels must be in 1..65535, height and width in 1..32767";
        return DGS_ERR_INVALID_ARG;
    }
    if (!(lambda >= 0.0f && lambda <= 1.0f)) {
        c->err = "loss: lambda must be in [0, 1]";
        return DGS_ERR_INVALID_ARG;
    }
    if (!image || !target || !loss) {
        c->err = "loss: NULL image, target or loss pointer";
        return DGS_ERR_INVALID_ARG;
    }
    hipSetDevice(c->device);
    const int64_t n = (int64_t)channels * height * width;
    const dim3 grid((unsigned)((width + kTileW - 1) / kTileW), (unsigned)((height + kTileH - 1) / kTileH),
                    (unsigned)channels);
    const int64_t tiles = (int64_t)grid.x * grid.y * grid.z;
    hipError_t e = ensure_buf(c->loss_part, c->cap_loss_part, 2 * tiles, c->stream);
    if (e == hipSuccess && grad_image) e = ensure_buf(c->loss_coef, c->cap_loss_coef, 3 * n, c->stream);
    if (e != hipSuccess) {
        c->err = std::string("loss: hipMalloc failed: ") + hipGetErrorString(e);
        return DGS_ERR_OOM;
    }
    LossArgs a;
    a.x = image;
    a.y = target;
    a.C = channels;
    a.H = height;
    a.W = width;
    a.lam = lambda;
    a.dls = (float)(-(double)lambda / (double)n);
    a.l1c = (float)((1.0 - (double)lambda) / (double)n);
    a.coef = grad_image ? c->loss_coef : nullptr;
    a.part = c->loss_part;
    a.grad = grad_image;
    const Window w = make_window();
    hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(kThreads), 0, c->stream, a, w);
    hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(kThreads), 0, c->stream, (const double*)c->loss_part,
                       (size_t)tiles, (double)n, (double)lambda, loss);
    if (grad_image) hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(kThreads), 0, c->stream, a, w);
    e = hipGetLastError();
    if (e != hipSuccess) {
        c->err = std::string("loss: kernel launch failed: ") + hipGetErrorString(e);
        return DGS_ERR_DEVICE;
    }
    return DGS_OK;
}

}  // extern "C"
