// Cell preprocessing and Gaussian projection (Duplex-GS Sec. IV-B, V-A, VI-A).
//
// Discrete decisions (near cull, depth key, pixel rectangles) are taken in
// binary32 with contraction off, correctly rounded division and square root
// and one fixed operation order, so that they are reproducible bit for bit.
// Continuous quantities (the projected mean, the conic, colour, v_n) feed
// the compositor; the projected mean is formed in binary64 and stored
// relative to the Gaussian's pixel rectangle so that the per-pixel offset
// keeps full precision at 4K.
#include "common.h"
#include "launch.h"

namespace dgs {

// ---------------------------------------------------------------- discrete

__device__ inline void view32(const CamK& k, float px, float py, float pz, float* o) {
#pragma clang fp contract(off)
    for (int i = 0; i < 3; i++)
        o[i] = ((k.R[i * 3 + 0] * px + k.R[i * 3 + 1] * py) + k.R[i * 3 + 2] * pz) + k.t[i];
}

// Screen covariance (xx, xy, yy) of a 3D Gaussian with scales s and
// quaternion q (w, x, y, z) whose camera-space centre is tc: local affine
// approximation of the perspective map (EWA splatting).
__device__ inline void ewa32(const CamK& k, const float* tc, float s0, float s1, float s2, float qw, float qx,
                             float qy, float qz, float* cov) {
#pragma clang fp contract(off)
    float n = sqrtf(((qw * qw + qx * qx) + qy * qy) + qz * qz);
    float w = qw / n, x = qx / n, y = qy / n, z = qz / n;
    float xx = x * x, yy = y * y, zz = z * z;
    float xy = x * y, xz = x * z, yz = y * z;
    float wx = w * x, wy = w * y, wz = w * z;
    float R[9];
    R[0] = 1.0f - 2.0f * (yy + zz); R[1] = 2.0f * (xy - wz);        R[2] = 2.0f * (xz + wy);
    R[3] = 2.0f * (xy + wz);        R[4] = 1.0f - 2.0f * (xx + zz); R[5] = 2.0f * (yz - wx);
    R[6] = 2.0f * (xz - wy);        R[7] = 2.0f * (yz + wx);        R[8] = 1.0f - 2.0f * (xx + yy);
    float M[9];
    for (int i = 0; i < 3; i++) {
        M[i * 3 + 0] = R[i * 3 + 0] * s0;
        M[i * 3 + 1] = R[i * 3 + 1] * s1;
        M[i * 3 + 2] = R[i * 3 + 2] * s2;
    }
    float S[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            S[i * 3 + j] = (M[i * 3 + 0] * M[j * 3 + 0] + M[i * 3 + 1] * M[j * 3 + 1]) + M[i * 3 + 2] * M[j * 3 + 2];
    float limx = 1.3f * ((0.5f * (float)k.W) / k.fx);
    float limy = 1.3f * ((0.5f * (float)k.H) / k.fy);
    float tz = tc[2];
    float txz = tc[0] / tz, tyz = tc[1] / tz;
    float txc = fminf(limx, fmaxf(-limx, txz)) * tz;
    float tyc = fminf(limy, fmaxf(-limy, tyz)) * tz;
    float tz2 = tz * tz;
    float j00 = k.fx / tz, j02 = -(k.fx * txc) / tz2;
    float j11 = k.fy / tz, j12 = -(k.fy * tyc) / tz2;
    float m0[3], m1[3];
    for (int j = 0; j < 3; j++) {
        m0[j] = j00 * k.R[0 * 3 + j] + j02 * k.R[2 * 3 + j];
        m1[j] = j11 * k.R[1 * 3 + j] + j12 * k.R[2 * 3 + j];
    }
    float w0[3], w1[3];
    for (int j = 0; j < 3; j++) {
        w0[j] = (m0[0] * S[0 * 3 + j] + m0[1] * S[1 * 3 + j]) + m0[2] * S[2 * 3 + j];
        w1[j] = (m1[0] * S[0 * 3 + j] + m1[1] * S[1 * 3 + j]) + m1[2] * S[2 * 3 + j];
    }
    cov[0] = (w0[0] * m0[0] + w0[1] * m0[1]) + w0[2] * m0[2];
    cov[1] = (w0[0] * m1[0] + w0[1] * m1[1]) + w0[2] * m1[2];
    cov[2] = (w1[0] * m1[0] + w1[1] * m1[1]) + w1[2] * m1[2];
}

__device__ inline float proj_x32(const CamK& k, const float* tc) {
#pragma clang fp contract(off)
    return k.fx * (tc[0] / tc[2]) + k.cx;
}
__device__ inline float proj_y32(const CamK& k, const float* tc) {
#pragma clang fp contract(off)
    return k.fy * (tc[1] / tc[2]) + k.cy;
}

// Pixels whose centres px + 0.5 lie in [u - h, u + h], clipped to the image.
__device__ inline bool rect32(const CamK& k, float ux, float uy, float hx, float hy, int* r) {
#pragma clang fp contract(off)
    float x0 = ceilf((ux - hx) - 0.5f), x1 = floorf((ux + hx) - 0.5f);
    float y0 = ceilf((uy - hy) - 0.5f), y1 = floorf((uy + hy) - 0.5f);
    if (!(x0 <= x1) || !(y0 <= y1)) return false;
    x0 = fmaxf(x0, 0.0f); x1 = fminf(x1, (float)(k.W - 1));
    y0 = fmaxf(y0, 0.0f); y1 = fminf(y1, (float)(k.H - 1));
    if (!(x0 <= x1) || !(y0 <= y1)) return false;
    r[0] = (int)x0; r[1] = (int)x1; r[2] = (int)y0; r[3] = (int)y1;
    return true;
}

// ---------------------------------------------------------------- continuous

// Real spherical harmonics (Condon-Shortley phase, m = -l..l) at the unit
// direction (x, y, z), dotted with planar coefficients c[j * stride].
__device__ inline float sh_eval(int deg, float x, float y, float z, const float* c, int64_t stride) {
    float s = 0.28209479177387814f * c[0];  // 0.5 sqrt(1/pi)
    if (deg < 1) return s;
    const float c1 = 0.4886025119029199f;   // sqrt(3/(4 pi))
    s += -c1 * y * c[stride] + c1 * z * c[2 * stride] - c1 * x * c[3 * stride];
    if (deg < 2) return s;
    float xx = x * x, yy = y * y, zz = z * z;
    s += 1.0925484305920792f * x * y * c[4 * stride];               // 0.5 sqrt(15/pi)
    s += -1.0925484305920792f * y * z * c[5 * stride];
    s += 0.31539156525252005f * (2.0f * zz - xx - yy) * c[6 * stride];  // 0.25 sqrt(5/pi)
    s += -1.0925484305920792f * x * z * c[7 * stride];
    s += 0.5462742152960396f * (xx - yy) * c[8 * stride];           // 0.25 sqrt(15/pi)
    if (deg < 3) return s;
    s += -0.5900435899266435f * y * (3.0f * xx - yy) * c[9 * stride];        // 0.125 sqrt(70/pi)
    s += 2.890611442640554f * x * y * z * c[10 * stride];                    // 0.5 sqrt(105/pi)
    s += -0.4570457994644658f * y * (4.0f * zz - xx - yy) * c[11 * stride];  // 0.125 sqrt(42/pi)
    s += 0.3731763325901154f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy) * c[12 * stride];  // 0.25 sqrt(7/pi)
    s += -0.4570457994644658f * x * (4.0f * zz - xx - yy) * c[13 * stride];
    s += 1.445305721320277f * z * (xx - yy) * c[14 * stride];                // 0.25 sqrt(105/pi)
    s += -0.5900435899266435f * x * (xx - 3.0f * yy) * c[15 * stride];
    return s;
}

__device__ inline void unit_dir(const CamK& k, float px, float py, float pz, float* d) {
    float x = px - k.o[0], y = py - k.o[1], z = pz - k.o[2];
    float inv = 1.0f / sqrtf(x * x + y * y + z * z);
    d[0] = x * inv; d[1] = y * inv; d[2] = z * inv;
}

// ---------------------------------------------------------------- kernels

// a1: one thread per cell.  Outputs the camera-depth key bits, the packed
// pixel rectangle of the kappa-sigma proxy box padded by 3 sqrt(delta), the
// number of tiles it touches (0 = culled) and v_n.  With CSR offsets it also
// checks the cell's member range (start >= 0, count in 0..kmax, end <= M,
// offs[0] = 0, offs[N] = M): a cell that breaks it is culled (no keys, so no
// walk reads its members) and the device error flag is set.
__global__ __launch_bounds__(256) void k_cell_preprocess(int N, const float* __restrict__ pos,
                                                         const float* __restrict__ scale,
                                                         const float* __restrict__ rot,
                                                         const float* __restrict__ vsh, int vdeg,
                                                         const int32_t* __restrict__ offs, int M, int kmax,
                                                         const FrameK* __restrict__ fr,
                                                         uint32_t* __restrict__ depth_bits,
                                                         uint64_t* __restrict__ prect,
                                                         uint32_t* __restrict__ ntiles, float* __restrict__ v_out,
                                                         int* __restrict__ err) {
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const CamK k = fr->k;
    const OptK o = fr->o;
    bool members_ok = true;
    if (offs) {
        const int a0 = offs[n], a1 = offs[n + 1];
        members_ok = a0 >= 0 && a1 >= a0 && a1 - a0 <= kmax && a1 <= M && (n > 0 || a0 == 0) &&
                     (n < N - 1 || a1 == M);
        if (!members_ok) atomicOr(err, 1 << kErrInvalid);
    }
    float p0 = pos[n], p1 = pos[N + n], p2 = pos[2 * N + n];
    float tc[3];
    view32(k, p0, p1, p2, tc);
    depth_bits[n] = __float_as_uint(tc[2]);
    uint64_t pr = kEmptyRect;
    uint32_t nt = 0;
    if (members_ok && tc[2] > k.znear) {
        float cov[3];
        ewa32(k, tc, scale[n], scale[N + n], scale[2 * N + n], rot[n], rot[N + n], rot[2 * N + n], rot[3 * N + n],
              cov);
        float ux = proj_x32(k, tc), uy = proj_y32(k, tc);
        float hx, hy;
        {
#pragma clang fp contract(off)
            float pad = 3.0f * sqrtf(o.delta);
            hx = o.kappa * sqrtf(cov[0]) + pad;
            hy = o.kappa * sqrtf(cov[2]) + pad;
        }
        int r[4];
        if (rect32(k, ux, uy, hx, hy, r)) {
            pr = pack_rect(r[0], r[1], r[2], r[3]);
            nt = (uint32_t)((r[1] / kTile - r[0] / kTile + 1) * (r[3] / kTile - r[2] / kTile + 1));
        }
    }
    prect[n] = pr;
    ntiles[n] = nt;
    float v = 1.0f;
    if (!o.v_one) {
        float d[3];
        unit_dir(k, p0, p1, p2, d);
        float s = sh_eval(vdeg, d[0], d[1], d[2], vsh + n, N);
        v = 1.0f / (1.0f + __expf(-s));
    }
    if (o.tau > 0.0f) v *= fmaxf(0.0f, 1.0f - tc[2] / o.tau);  // LC-WSR weight of the cell
    v_out[n] = v;
}

// a2 for Gaussian g.  In Duplex mode only members of cells that survived a1
// are projected (cell_ntiles != null); every Gaussian gets its packed pixel
// rectangle (kEmptyRect when culled), projected ones a GRec.  In alpha mode
// (cell_ntiles == null) it also writes the depth key bits and tile count
// used for per-Gaussian keys.
__device__ inline void gauss_project_one(
    int g, int M, int K, const float* __restrict__ means, const float* __restrict__ scales,
    const float* __restrict__ rots, const float* __restrict__ opac, const float* __restrict__ sh, int sh_deg,
    const FrameK* __restrict__ fr, const uint32_t* __restrict__ cell_ntiles, GRec* __restrict__ recs,
    uint64_t* __restrict__ grect, uint32_t* __restrict__ gdepth, uint32_t* __restrict__ gntiles) {
    const CamK k = fr->k;
    const OptK o = fr->o;
    if (cell_ntiles && cell_ntiles[g / K] == 0) {
        grect[g] = kEmptyRect;
        return;
    }
    float m0 = means[g], m1 = means[M + g], m2 = means[2 * M + g];
    float sg = opac[g];
    float tc[3];
    view32(k, m0, m1, m2, tc);
    int r[4];
    bool vis = false;
    float cov[3];
    if (sg > 0.0f && tc[2] > k.znear) {
        ewa32(k, tc, scales[g], scales[M + g], scales[2 * M + g], rots[g], rots[M + g], rots[2 * M + g],
              rots[3 * M + g], cov);
        float a, c, hx, hy;
        {
#pragma clang fp contract(off)
            a = cov[0] + o.delta;
            c = cov[2] + o.delta;
            hx = 3.0f * sqrtf(a);
            hy = 3.0f * sqrtf(c);
        }
        cov[0] = a;
        cov[2] = c;
        vis = rect32(k, proj_x32(k, tc), proj_y32(k, tc), hx, hy, r);
    }
    if (gdepth) {
        gdepth[g] = __float_as_uint(tc[2]);
        gntiles[g] = vis ? (uint32_t)((r[1] / kTile - r[0] / kTile + 1) * (r[3] / kTile - r[2] / kTile + 1)) : 0u;
    }
    if (!vis) {
        grect[g] = kEmptyRect;
        GRec e = {};
        e.x0 = 0x7fff0000;
        e.y0 = 0x7fff0000;
        e.wxy = 0;
        recs[g] = e;
        return;
    }
    grect[g] = pack_rect(r[0], r[1], r[2], r[3]);
    // projected mean in binary64, stored as an offset from the rectangle corner
    double tx = k.Rd[0] * m0 + k.Rd[1] * m1 + k.Rd[2] * m2 + k.td[0];
    double ty = k.Rd[3] * m0 + k.Rd[4] * m1 + k.Rd[5] * m2 + k.td[1];
    double tz = k.Rd[6] * m0 + k.Rd[7] * m1 + k.Rd[8] * m2 + k.td[2];
    double ux = (double)k.fx * (tx / tz) + (double)k.cx;
    double uy = (double)k.fy * (ty / tz) + (double)k.cy;
    GRec e;
    e.ox = (float)(((double)r[0] + 0.5) - ux);
    e.oy = (float)(((double)r[2] + 0.5) - uy);
    float det = cov[0] * cov[2] - cov[1] * cov[1];
    const float l2e = 1.4426950408889634f;
    e.ca = -0.5f * l2e * cov[2] / det;
    e.cb = l2e * cov[1] / det;   // -log2e * (-b / det)
    e.cc = -0.5f * l2e * cov[0] / det;
    e.lo = __log2f(sg);
    float d[3];
    unit_dir(k, m0, m1, m2, d);
    int64_t cs = 3 * (int64_t)M;
    float cr, cg, cb;
    if (sh_deg < 0) {  // decoded Gaussians: colour given directly, planar [3][M]
        cr = sh[g];
        cg = sh[M + g];
        cb = sh[2 * (int64_t)M + g];
    } else {
        cr = 0.5f + sh_eval(sh_deg, d[0], d[1], d[2], sh + g, cs);
        cg = 0.5f + sh_eval(sh_deg, d[0], d[1], d[2], sh + M + g, cs);
        cb = 0.5f + sh_eval(sh_deg, d[0], d[1], d[2], sh + 2 * (int64_t)M + g, cs);
    }
    e.r = fmaxf(cr, 0.0f);
    e.g = fmaxf(cg, 0.0f);
    e.b = fmaxf(cb, 0.0f);
    e.x0 = r[0];
    e.y0 = r[2];
    e.wxy = (uint32_t)(r[1] - r[0]) | ((uint32_t)(r[3] - r[2]) << 16);
    recs[g] = e;
}

// Grid-stride over the Gaussians.  When the projection runs beside the cell
// sort (on a second stream) its grid is capped, so that the sort's small
// latency-bound grids still find free CUs.
constexpr int kOverlapProjectBlocks = 1024;

__global__ __launch_bounds__(256) void k_gauss_project(
    int M, int K, const float* __restrict__ means, const float* __restrict__ scales,
    const float* __restrict__ rots, const float* __restrict__ opac, const float* __restrict__ sh, int sh_deg,
    const FrameK* __restrict__ fr, const uint32_t* __restrict__ cell_ntiles, GRec* __restrict__ recs,
    uint64_t* __restrict__ grect, uint32_t* __restrict__ gdepth, uint32_t* __restrict__ gntiles) {
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < M; g += gridDim.x * blockDim.x)
        gauss_project_one(g, M, K, means, scales, rots, opac, sh, sh_deg, fr, cell_ntiles, recs, grect, gdepth, gntiles);
}

void launch_cell_preprocess(hipStream_t st, int N, const float* pos, const float* scale, const float* rot,
                            const float* vsh, int vdeg, const int32_t* offs, int M, int kmax, const FrameK* fr,
                            uint32_t* depth_bits, uint64_t* prect, uint32_t* ntiles, float* v, int* err) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_cell_preprocess, dim3((N + 255) / 256), dim3(256), 0, st, N, pos, scale, rot, vsh, vdeg,
                       offs, M, kmax, fr, depth_bits, prect, ntiles, v, err);
}

void launch_gauss_project(hipStream_t st, int M, int K, const float* means, const float* scales,
                          const float* rots, const float* opac, const float* sh, int sh_deg, const FrameK* fr,
                          const uint32_t* cell_ntiles, GRec* recs, uint64_t* grect, uint32_t* gdepth,
                          uint32_t* gntiles, bool overlapped) {
    if (M <= 0) return;
    const int blocks = (M + 255) / 256, cap = overlapped ? kOverlapProjectBlocks : blocks;
    hipLaunchKernelGGL(k_gauss_project, dim3(blocks < cap ? blocks : cap), dim3(256), 0, st, M, K, means, scales, rots, opac,
                       sh, sh_deg, fr, cell_ntiles, recs, grect, gdepth, gntiles);
}

__global__ void k_set_frame(FrameK f, FrameK* dst) {
    if (threadIdx.x == 0) *dst = f;
}

void launch_set_frame(hipStream_t st, const FrameK& f, FrameK* dst) {
    hipLaunchKernelGGL(k_set_frame, dim3(1), dim3(64), 0, st, f, dst);
}

}  // namespace dgs
