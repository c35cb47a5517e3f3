// Neural decode of cells (Sec. III-A neural Gaussians; Sec. IV-A cell
// proxy): each cell's K Gaussians come from its latent feature f_n, the
// viewing distance delta_n and direction d_n through four two-layer MLPs
// F_sigma (tanh), F_c (sigmoid), F_s (sigmoid scale ratio) and F_q (raw
// quaternion); centres follow eq. scaffold_offset with the offsets in the
// cell frame, mu = x_n + R(Q_n)(O^pos * S_n), and scales eqs. nerual_scales
// and scale_res, s = max(0, min(sigmoid(y_s), 1 - |O^pos|)) * S_n.
//
// Mapping: one decoder per workgroup (blockIdx.y), one cell per thread, so
// all lanes read the same weight at the same time and it comes through a
// scalar load; each thread writes its decoder's attribute of the cell's
// Gaussians straight to the planar outputs.  The opacity decoder, whose
// second layer is the smallest, also places the centres.  F = H = 32 (the
// neural-Gaussian default) has an exact-size kernel whose first layer runs
// input-major over contiguous weight rows; other sizes use register
// capacities of 36 x 32 or 68 x 64 with predicated loops (the largest
// spills to scratch).
//
// The scales, quaternions and centres decide each Gaussian's pixel box, so
// they are computed in binary32 in one fixed order: every sum is a chain of
// fused multiply-adds in ascending index order starting from the bias, the
// sigmoid uses the exp below, and no other contraction happens.  Opacity and
// colour only enter the continuous layer.
#include "common.h"
#include "launch.h"

namespace dgs {

// exp(x) in binary32: Cody-Waite reduction x = n ln2 + r with ln2 split so
// that n * ln2_hi is exact, the degree-7 Taylor polynomial of e^r in Horner
// form, then the exact scaling by 2^n; one rounding per operation.
__device__ inline float exp32_def(float x) {
#pragma clang fp contract(off)
    x = fminf(88.0f, fmaxf(-88.0f, x));
    const float log2e = 1.44269504088896341f;
    const float ln2_hi = 0.693145751953125f, ln2_lo = 1.42860682030941723e-6f;
    const float n = rintf(x * log2e);
    const float r = (x - n * ln2_hi) - n * ln2_lo;
    float p = 1.0f / 5040.0f;
    p = p * r + 1.0f / 720.0f;
    p = p * r + 1.0f / 120.0f;
    p = p * r + 1.0f / 24.0f;
    p = p * r + 1.0f / 6.0f;
    p = p * r + 0.5f;
    p = p * r + 1.0f;
    p = p * r + 1.0f;
    return ldexpf(p, (int)n);
}

__device__ inline float sigmoid32_def(float y) {
#pragma clang fp contract(off)
    return 1.0f / (1.0f + exp32_def(-y));
}

// Rotation of a cell quaternion (w, x, y, z), normalised first.
__device__ inline void cell_rot32(float w, float x, float y, float z, float* R) {
#pragma clang fp contract(off)
    const float n = sqrtf(((w * w + x * x) + y * y) + z * z);
    w = w / n; x = x / n; y = y / n; z = z / n;
    const float xx = x * x, yy = y * y, zz = z * z;
    const float xy = x * y, xz = x * z, yz = y * z;
    const float wx = w * x, wy = w * y, wz = w * z;
    R[0] = 1.0f - 2.0f * (yy + zz); R[1] = 2.0f * (xy - wz);        R[2] = 2.0f * (xz + wy);
    R[3] = 2.0f * (xy + wz);        R[4] = 1.0f - 2.0f * (xx + zz); R[5] = 2.0f * (yz - wx);
    R[6] = 2.0f * (xz - wy);        R[7] = 2.0f * (yz + wx);        R[8] = 1.0f - 2.0f * (xx + yy);
}

// CI, CH: register capacities of the input vector and the hidden layer (the
// loops run over them, predicated by the actual sizes, so the arrays stay in
// registers and every sum keeps its order).
template <int CI, int CH>
__global__ __launch_bounds__(256) void k_decode(DecodeArgs a) {
#pragma clang fp contract(off)
    const int wave = blockIdx.y;  // the decoder
    const int n = blockIdx.x * 256 + threadIdx.x;
    const int N = a.N, K = a.K, F = a.F, H = a.H, I = a.F + 4;
    const bool live = n < N && (a.cell_ntiles == nullptr || a.cell_ntiles[n] != 0);
    if (!__any(live)) return;  // uniform per wavefront
    const CamK& k = a.fr->k;
    const int64_t M = (int64_t)N * K;

    // input vector (f, delta, d) and the layer-1 activations in registers
    float x[CI], h[CH];
    float px = 0.0f, py = 0.0f, pz = 0.0f, ex = 0.0f, ey = 0.0f, ez = 0.0f, dist = 1.0f;
    if (live) {
        px = a.cell_pos[n];
        py = a.cell_pos[N + n];
        pz = a.cell_pos[2 * N + n];
        ex = px - k.o[0];
        ey = py - k.o[1];
        ez = pz - k.o[2];
        dist = sqrtf((ex * ex + ey * ey) + ez * ez);
    }
#pragma unroll
    for (int i = 0; i < CI; i++) {
        float v = 0.0f;
        if (i < F) v = live ? a.features[(int64_t)i * N + n] : 0.0f;
        else if (i == F) v = dist;
        else if (i == F + 1) v = ex / dist;
        else if (i == F + 2) v = ey / dist;
        else if (i == F + 3) v = ez / dist;
        x[i] = v;
    }
    const int A = wave == 0 ? 1 : wave == 3 ? 4 : 3;  // outputs per Gaussian of this decoder
    const float* w = a.weights + a.woff[wave];
    const float* W1 = w;
    const float* b1 = W1 + (int64_t)I * H;
    const float* W2 = b1 + H;
    const int O = K * A;
    const float* b2 = W2 + (int64_t)H * O;
#pragma unroll
    for (int j = 0; j < CH; j++) {
        float acc = 0.0f;
        if (j < H) {
            acc = b1[j];
#pragma unroll
            for (int i = 0; i < CI; i++)
                if (i < I) acc = fmaf(x[i], W1[(int64_t)i * H + j], acc);
        }
        h[j] = acc > 0.0f ? acc : 0.0f;
    }
    if (!live) return;
    const float S[3] = {a.cell_scale[n], a.cell_scale[N + n], a.cell_scale[2 * N + n]};
    for (int kk = 0; kk < K; kk++) {
        const int64_t g = (int64_t)n * K + kk;
        float y[4];
#pragma unroll
        for (int c = 0; c < 4; c++) {
            float acc = 0.0f;
            if (c < A) {
                const int o = kk * A + c;
                acc = b2[o];
#pragma unroll
                for (int j = 0; j < CH; j++)
                    if (j < H) acc = fmaf(h[j], W2[(int64_t)j * O + o], acc);
            }
            y[c] = acc;
        }
        if (wave == 0) {
            a.opac[g] = tanhf(y[0]);
            // centre in the cell frame
            float R[9];
            cell_rot32(a.cell_rot[n], a.cell_rot[N + n], a.cell_rot[2 * N + n], a.cell_rot[3 * N + n], R);
            const float u0 = a.offsets[g] * S[0], u1 = a.offsets[M + g] * S[1], u2 = a.offsets[2 * M + g] * S[2];
            a.means[g] = px + ((R[0] * u0 + R[1] * u1) + R[2] * u2);
            a.means[M + g] = py + ((R[3] * u0 + R[4] * u1) + R[5] * u2);
            a.means[2 * M + g] = pz + ((R[6] * u0 + R[7] * u1) + R[8] * u2);
        } else if (wave == 1) {
#pragma unroll
            for (int c = 0; c < 3; c++) a.color[c * M + g] = 1.0f / (1.0f + __expf(-y[c]));
        } else if (wave == 2) {
            const float o0 = a.offsets[g], o1 = a.offsets[M + g], o2 = a.offsets[2 * M + g];
            const float lim = 1.0f - sqrtf((o0 * o0 + o1 * o1) + o2 * o2);
#pragma unroll
            for (int c = 0; c < 3; c++) {
                float r = sigmoid32_def(y[c]);
                r = r < lim ? r : lim;
                r = r > 0.0f ? r : 0.0f;
                a.scales[c * M + g] = r * S[c];
            }
        } else {
#pragma unroll
            for (int c = 0; c < 4; c++) a.rots[c * M + g] = y[c];
        }
    }
}

// Exact-size variant (F, H known at compile time): layer 1 runs input-major
// (every weight row is one contiguous scalar load) and layer 2 reads, per
// hidden unit, the A contiguous outputs of one member.  Each sum keeps the
// order of the general kernel: bias first, then ascending index.
struct DecodeOut {
    float* __restrict__ means;
    float* __restrict__ scales;
    float* __restrict__ rots;
    float* __restrict__ opac;
    float* __restrict__ color;
};

template <int F, int H, int A>
__device__ inline void decode_wave(const DecodeArgs& a, const float* __restrict__ w, const float (&x)[F + 4],
                                   bool live, int n, float px, float py, float pz, int wave, const DecodeOut& out) {
#pragma clang fp contract(off)
    constexpr int I = F + 4;
    const int K = a.K, N = a.N;
    const int O = K * A;
    const float* W1 = w;
    const float* b1 = W1 + I * H;
    const float* W2 = b1 + H;
    const float* b2 = W2 + (int64_t)H * O;
    float h[H];
#pragma unroll
    for (int j = 0; j < H; j++) h[j] = b1[j];
#pragma unroll
    for (int i = 0; i < I; i++) {
        const float xi = x[i];
#pragma unroll
        for (int j = 0; j < H; j++) h[j] = fmaf(xi, W1[i * H + j], h[j]);
    }
#pragma unroll
    for (int j = 0; j < H; j++) h[j] = h[j] > 0.0f ? h[j] : 0.0f;
    // every lane stays in the loop (uniform control flow keeps the weight
    // loads scalar); only live lanes store
    const int64_t M = (int64_t)N * K;
    const int nn = live ? n : 0;
    const float S[3] = {a.cell_scale[nn], a.cell_scale[N + nn], a.cell_scale[2 * N + nn]};
    for (int kk = 0; kk < K; kk++) {
        const int64_t g = (int64_t)n * K + kk;
        float y[A];
#pragma unroll
        for (int c = 0; c < A; c++) y[c] = b2[kk * A + c];
#pragma unroll
        for (int j = 0; j < H; j++) {
#pragma unroll
            for (int c = 0; c < A; c++) y[c] = fmaf(h[j], W2[(int64_t)j * O + kk * A + c], y[c]);
        }
        if (!live) continue;
        if (wave == 0) {
            out.opac[g] = tanhf(y[0]);
            float R[9];
            cell_rot32(a.cell_rot[n], a.cell_rot[N + n], a.cell_rot[2 * N + n], a.cell_rot[3 * N + n], R);
            const float u0 = a.offsets[g] * S[0], u1 = a.offsets[M + g] * S[1], u2 = a.offsets[2 * M + g] * S[2];
            out.means[g] = px + ((R[0] * u0 + R[1] * u1) + R[2] * u2);
            out.means[M + g] = py + ((R[3] * u0 + R[4] * u1) + R[5] * u2);
            out.means[2 * M + g] = pz + ((R[6] * u0 + R[7] * u1) + R[8] * u2);
        } else if (wave == 1) {
#pragma unroll
            for (int c = 0; c < A; c++) out.color[c * M + g] = 1.0f / (1.0f + __expf(-y[c]));
        } else if (wave == 2) {
            const float o0 = a.offsets[g], o1 = a.offsets[M + g], o2 = a.offsets[2 * M + g];
            const float lim = 1.0f - sqrtf((o0 * o0 + o1 * o1) + o2 * o2);
#pragma unroll
            for (int c = 0; c < A; c++) {
                float r = sigmoid32_def(y[c]);
                r = r < lim ? r : lim;
                r = r > 0.0f ? r : 0.0f;
                out.scales[c * M + g] = r * S[c];
            }
        } else {
#pragma unroll
            for (int c = 0; c < A; c++) out.rots[c * M + g] = y[c];
        }
    }
}

template <int F, int H>
__global__ __launch_bounds__(256) void k_decode_exact(DecodeArgs a, const float* __restrict__ weights,
                                                      float* __restrict__ means, float* __restrict__ scales,
                                                      float* __restrict__ rots, float* __restrict__ opac,
                                                      float* __restrict__ color) {
#pragma clang fp contract(off)
    // one decoder per workgroup (blockIdx.y), one cell per thread: the
    // wavefronts of a compute unit mostly run the same code
    const int wave = blockIdx.y;
    const int n = blockIdx.x * 256 + threadIdx.x;
    const int N = a.N;
    const bool live = n < N && (a.cell_ntiles == nullptr || a.cell_ntiles[n] != 0);
    if (!__any(live)) return;  // uniform per wavefront
    const CamK& k = a.fr->k;
    float x[F + 4];
    float px = 0.0f, py = 0.0f, pz = 0.0f, ex = 0.0f, ey = 0.0f, ez = 0.0f, dist = 1.0f;
    if (live) {
        px = a.cell_pos[n];
        py = a.cell_pos[N + n];
        pz = a.cell_pos[2 * N + n];
        ex = px - k.o[0];
        ey = py - k.o[1];
        ez = pz - k.o[2];
        dist = sqrtf((ex * ex + ey * ey) + ez * ez);
    }
#pragma unroll
    for (int i = 0; i < F; i++) x[i] = live ? a.features[(int64_t)i * N + n] : 0.0f;
    x[F] = dist;
    x[F + 1] = ex / dist;
    x[F + 2] = ey / dist;
    x[F + 3] = ez / dist;
    const DecodeOut out{means, scales, rots, opac, color};
    const float* __restrict__ w = weights + a.woff[wave];
    if (wave == 0)
        decode_wave<F, H, 1>(a, w, x, live, n, px, py, pz, wave, out);
    else if (wave == 3)
        decode_wave<F, H, 4>(a, w, x, live, n, px, py, pz, wave, out);
    else
        decode_wave<F, H, 3>(a, w, x, live, n, px, py, pz, wave, out);
}

void launch_decode(hipStream_t st, const DecodeArgs& a) {
    if (a.N <= 0) return;
    const dim3 grid((unsigned)((a.N + 255) / 256), 4);
    if (a.F == 32 && a.H == 32)
        hipLaunchKernelGGL((k_decode_exact<32, 32>), grid, dim3(256), 0, st, a, a.weights, a.means, a.scales, a.rots,
                           a.opac, a.color);
    else if (a.F <= 32 && a.H <= 32)
        hipLaunchKernelGGL((k_decode<36, 32>), grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_decode<kMaxFeature + 4, kMaxHidden>), grid, dim3(256), 0, st, a);
}

}  // namespace dgs
