// Training loss of eq. `loss` without its perceptual term,
//     L = (1 - lam) mean |x - y| + lam (1 - mean SSIM(x, y)),
// and dL/dx, for planar [C][H][W] binary32 images (lam = lambda_1 = 0.2 in
// the paper's experimental settings).  SSIM per channel from an 11 x 11
// Gaussian window (sigma 1.5, weights summing to 1), the image zero outside
// its borders, c1 = 0.01^2, c2 = 0.03^2.
//
// Two passes, each streaming down strips of 64 columns: a wavefront owns
// one strip (lane l: column c0 + l) and kRowsOut output rows; it walks the
// kRowsOut + 10 input rows top to bottom, loading each row (with the
// 5-column halo on either side) a few rows ahead, blurs it along the row
// from a per-wavefront LDS row buffer, and keeps the last 11 row sums in
// registers for the blur along the column -- no workgroup barriers, no
// 2D tile in LDS:
//   k_ssim_fwd  window statistics of x and y -> the SSIM map; per-strip sums
//               of SSIM and |x - y| (binary64) and, when a gradient is
//               wanted, the three per-pixel coefficients of dL/dx:
//               dL/d mu_x, dL/d E[x^2], dL/d E[xy];
//   k_ssim_bwd  dL/dx = blur(dL/d mu_x) + 2 x blur(dL/d E[x^2])
//               + y blur(dL/d E[xy]) + (1 - lam)/n sign(x - y)
//               (the window is symmetric, so the adjoint of the zero-filled
//               blur is the same blur);
//   k_loss_sum  the strip sums in a fixed order -> L (binary64, stored as
//               binary32): the result does not depend on scheduling.
// Everything is HBM-bound: x and y are read twice, three coefficient planes
// written and read once, the gradient written once.
#include <math.h>

#include <string>

#include "ctx.h"

using namespace dgs;

namespace {

constexpr int kTaps = 11, kRad = 5;
constexpr int kStrip = 64;                    // columns per wavefront (one per lane)
constexpr int kWaves = 4;                     // strips side by side per workgroup
constexpr int kThreads = 64 * kWaves;
constexpr int kRowsOut = 32;                  // output rows per wavefront
constexpr int kRowsIn = kRowsOut + 2 * kRad;  // input rows it reads
constexpr int kAhead = 4;                     // input rows loaded ahead
constexpr int kRowBuf = kStrip + 2 * kRad + 6;  // one row and its halo (+ padding)
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

// Orders a wavefront's LDS row-buffer writes before its reads (and the
// reads before the next row's writes): the lanes exchange values through it.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A strip's columns: lane l reads column c0 - 5 + l, lanes below 10 also
// column c0 + 59 + l (the right halo); zero outside the image.
struct StripCols {
    int ca, cb;
    bool hb;
    __device__ __forceinline__ StripCols(int c0, int lane)
        : ca(c0 - kRad + lane), cb(c0 + kStrip - kRad + lane), hb(lane < 2 * kRad) {}
    __device__ __forceinline__ void load(const float* P, int H, int W, int gy, float& va, float& vb) const {
        const bool rin = gy >= 0 && gy < H;
        const size_t row = (size_t)(rin ? gy : 0) * W;
        va = rin && ca >= 0 && ca < W ? P[row + ca] : 0.0f;
        vb = rin && hb && cb < W ? P[row + cb] : 0.0f;
    }
};

// The part index of this wavefront's strip.
__device__ __forceinline__ size_t strip_index() {
    return (((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * kWaves + (threadIdx.x >> 6);
}

// The forward pass's state along one strip: rows in flight, the last 11
// row sums and centre values, the running sums.
struct FwdStrip {
    const float* X;
    const float* Y;
    float* bx;
    float* by;
    StripCols cols;
    int c, r0, gx, lane;
    size_t plane;
    float ax[kAhead], hx[kAhead], ay[kAhead], hy[kAhead];
    float ring[kTaps][5];                // row sums of x, y, x^2, y^2, xy of the last 11 rows
    float cxv[kRad + 1], cyv[kRad + 1];  // x, y at column c0 + lane of the last 6 rows
    double ssum, l1sum;
};

// Input row I of the strip (image row r0 - 5 + I); from I = 10 on, also
// output row r0 + I - 10 (centre row I - 5).  A template per row, so that
// every ring index is a constant (the rows are unrolled by the recursion).
template <int I>
__device__ __forceinline__ void fwd_row(FwdStrip& st, const LossArgs& a, const Window& w) {
    constexpr int sl = I % kAhead;
    wave_sync();  // the previous row's reads are done
    st.bx[st.lane] = st.ax[sl];
    st.by[st.lane] = st.ay[sl];
    if (st.cols.hb) {
        st.bx[kStrip + st.lane] = st.hx[sl];
        st.by[kStrip + st.lane] = st.hy[sl];
    }
    wave_sync();
    if constexpr (I + kAhead < kRowsIn) {
        st.cols.load(st.X, a.H, a.W, st.r0 - kRad + I + kAhead, st.ax[sl], st.hx[sl]);
        st.cols.load(st.Y, a.H, a.W, st.r0 - kRad + I + kAhead, st.ay[sl], st.hy[sl]);
    }
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f, s4 = 0.0f;
#pragma unroll
    for (int t = 0; t < kTaps; t++) {
        const float xv = st.bx[st.lane + t], yv = st.by[st.lane + t], g = w.g[t];
        s0 = fmaf(g, xv, s0);
        s1 = fmaf(g, yv, s1);
        s2 = fmaf(g, xv * xv, s2);
        s3 = fmaf(g, yv * yv, s3);
        s4 = fmaf(g, xv * yv, s4);
    }
    constexpr int rs = I % kTaps;
    st.ring[rs][0] = s0;
    st.ring[rs][1] = s1;
    st.ring[rs][2] = s2;
    st.ring[rs][3] = s3;
    st.ring[rs][4] = s4;
    st.cxv[I % (kRad + 1)] = st.bx[st.lane + kRad];
    st.cyv[I % (kRad + 1)] = st.by[st.lane + kRad];
    if constexpr (I >= 2 * kRad) {
        const int gy = st.r0 + I - 2 * kRad;
        if (gy < a.H && st.gx < a.W) {
            float m[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int k = 0; k < kTaps; k++) {
                const float g = w.g[k];
#pragma unroll
                for (int t = 0; t < 5; t++) m[t] = fmaf(g, st.ring[(I - 2 * kRad + k) % kTaps][t], m[t]);
            }
            const float mx = m[0], my = m[1];
            const float sxx = m[2] - mx * mx, syy = m[3] - my * my, sxy = m[4] - mx * my;
            const float a1 = 2.0f * mx * my + kC1, a2 = 2.0f * sxy + kC2;
            const float b1 = mx * mx + my * my + kC1, b2 = sxx + syy + kC2;
            const float sv = (a1 * a2) / (b1 * b2);
            constexpr int cs = (I - kRad) % (kRad + 1);
            st.ssum += (double)sv;
            st.l1sum += (double)fabsf(st.cxv[cs] - st.cyv[cs]);
            if (a.coef) {
                // S = a1 a2 / (b1 b2): d/d mu_x through a1 (2 mu_y), a2 (-2 mu_y),
                // b1 (2 mu_x), b2 (-2 mu_x); d/d E[x^2] through b2; d/d E[xy] through a2
                const float ds = a.dls * sv;
                const size_t p = st.c * st.plane + (size_t)gy * a.W + st.gx, n = (size_t)a.C * st.plane;
                a.coef[p] = ds * (2.0f * my / a1 - 2.0f * my / a2 - 2.0f * mx / b1 + 2.0f * mx / b2);
                a.coef[n + p] = -ds / b2;
                a.coef[2 * n + p] = 2.0f * ds / a2;
            }
        }
    }
    if constexpr (I + 1 < kRowsIn) fwd_row<I + 1>(st, a, w);
}

__global__ __launch_bounds__(kThreads) void k_ssim_fwd(LossArgs a, Window w) {
    __shared__ float rb[kWaves][2][kRowBuf];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int c = blockIdx.z;
    const int c0 = (blockIdx.x * kWaves + wv) * kStrip, r0 = blockIdx.y * kRowsOut;
    const size_t plane = (size_t)a.H * a.W;
    FwdStrip st{a.x + c * plane, a.y + c * plane, rb[wv][0], rb[wv][1], StripCols(c0, lane), c, r0, c0 + lane,
                lane, plane};
    st.ssum = 0.0;
    st.l1sum = 0.0;
    // input row i is image row r0 - 5 + i; rows i .. i + kAhead - 1 are in flight
#pragma unroll
    for (int i = 0; i < kAhead; i++) {
        st.cols.load(st.X, a.H, a.W, r0 - kRad + i, st.ax[i], st.hx[i]);
        st.cols.load(st.Y, a.H, a.W, r0 - kRad + i, st.ay[i], st.hy[i]);
    }
    fwd_row<0>(st, a, w);
    const double ssum = wave_sum(st.ssum), l1sum = wave_sum(st.l1sum);
    if (lane == 0) {
        const size_t t = strip_index();
        a.part[2 * t] = ssum;
        a.part[2 * t + 1] = l1sum;
    }
}

__global__ __launch_bounds__(kThreads) void k_ssim_bwd(LossArgs a, Window w) {
    __shared__ float rb[kWaves][3][kRowBuf];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int c = blockIdx.z;
    const int c0 = (blockIdx.x * kWaves + wv) * kStrip, r0 = blockIdx.y * kRowsOut;
    const size_t plane = (size_t)a.H * a.W, n = (size_t)a.C * plane;
    const float* cf[3] = {a.coef + c * plane, a.coef + n + c * plane, a.coef + 2 * n + c * plane};
    const StripCols cols(c0, lane);
    float av[kAhead][3], hv[kAhead][3];
#pragma unroll
    for (int i = 0; i < kAhead; i++)
#pragma unroll
        for (int q = 0; q < 3; q++) cols.load(cf[q], a.H, a.W, r0 - kRad + i, av[i][q], hv[i][q]);
    float ring[kTaps][3];  // row sums of the three coefficient planes of the last 11 rows
    const int gx = c0 + lane;
#pragma unroll
    for (int i = 0; i < kRowsIn; i++) {
        const int sl = i % kAhead;
        wave_sync();
#pragma unroll
        for (int q = 0; q < 3; q++) {
            rb[wv][q][lane] = av[sl][q];
            if (cols.hb) rb[wv][q][kStrip + lane] = hv[sl][q];
        }
        wave_sync();
        if (i + kAhead < kRowsIn) {
#pragma unroll
            for (int q = 0; q < 3; q++) cols.load(cf[q], a.H, a.W, r0 - kRad + i + kAhead, av[sl][q], hv[sl][q]);
        }
        float s[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t < kTaps; t++) {
            const float g = w.g[t];
#pragma unroll
            for (int q = 0; q < 3; q++) s[q] = fmaf(g, rb[wv][q][lane + t], s[q]);
        }
#pragma unroll
        for (int q = 0; q < 3; q++) ring[i % kTaps][q] = s[q];
        if (i < 2 * kRad) continue;
        const int gy = r0 + i - 2 * kRad;
        if (gy >= a.H || gx >= a.W) continue;
        float b[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < kTaps; k++) {
            const float g = w.g[k];
#pragma unroll
            for (int q = 0; q < 3; q++) b[q] = fmaf(g, ring[(i - 2 * kRad + k) % kTaps][q], b[q]);
        }
        const size_t p = c * plane + (size_t)gy * a.W + gx;
        const float xv = a.x[p], yv = a.y[p];
        const float sg = (float)(xv > yv) - (float)(xv < yv);
        a.grad[p] = fmaf(a.l1c, sg, fmaf(yv, b[2], fmaf(2.0f * xv, b[1], b[0])));
    }
}

// One workgroup: the strip sums in a fixed order, then L.
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
    const dim3 grid((unsigned)((width + kWaves * kStrip - 1) / (kWaves * kStrip)),
                    (unsigned)((height + kRowsOut - 1) / kRowsOut), (unsigned)channels);
    const int64_t tiles = (int64_t)grid.x * grid.y * grid.z * kWaves;  // strips
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
