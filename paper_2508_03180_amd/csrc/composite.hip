// Tile compositors.
//
// Duplex (Sec. V-A, eq. hybrid_renderer with w_n = v_n T_n, eq. dulpex_T;
// Sec. V-B early termination; Sec. VI-A false-positive skip).  For every
// pixel the cells of its tile are walked front to back.  Inside a cell the
// members are summed without order:
//     A = sum alpha c,  B = sum alpha,  P = prod (1 - v alpha)
// over members whose box contains the pixel and whose alpha reaches
// alpha_min, with alpha = min(alpha_max, sigma G'(x')).  Across cells
//     N += v T A,  D += v T B,  T *= P,
// a cell is blended only while T (the transmittance in front of it) is at
// least eps, and the colour is C = N / D (bg where D = 0).
//
// Alpha (eqs. alpha_blending, transmittance): the same walk over
// depth-sorted Gaussians with C += T alpha c, T *= 1 - alpha, plus T bg.
//
// One workgroup (4 wavefronts) per 16x16 tile; wavefront w owns the 8x8
// quadrant (w & 1, w >> 1), lane l the pixel (l & 7, l >> 3) in it.  Batches
// of up to 256 Gaussian records are staged in LDS together with a per-record
// and per-cell mask of the quadrants their boxes touch, so a wavefront skips
// whole cells and Gaussians that miss its quadrant.
#include "common.h"
#include "launch.h"

namespace dgs {

struct PixelCoord {
    int px, py;
    bool valid;
};

__device__ inline PixelCoord tile_pixel(int tile, int TX, int W, int H) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    PixelCoord c;
    c.px = (tile % TX) * kTile + (wave & 1) * 8 + (lane & 7);
    c.py = (tile / TX) * kTile + (wave >> 1) * 8 + (lane >> 3);
    c.valid = c.px < W && c.py < H;
    return c;
}

// Quadrant-overlap mask (bit w for wavefront w) of a record's box inside tile.
__device__ inline uint32_t quad_mask(const GRec& e, int tx0, int ty0) {
    const int wx = (int)(e.wxy & 0xffffu), wy = (int)(e.wxy >> 16);
    const int x0 = e.x0 - tx0, x1 = x0 + wx, y0 = e.y0 - ty0, y1 = y0 + wy;
    uint32_t m = 0;
    const bool c0 = x0 <= 7 && x1 >= 0, c1 = x0 <= 15 && x1 >= 8;
    const bool r0 = y0 <= 7 && y1 >= 0, r1 = y0 <= 15 && y1 >= 8;
    if (r0 && c0) m |= 1u;
    if (r0 && c1) m |= 2u;
    if (r1 && c0) m |= 4u;
    if (r1 && c1) m |= 8u;
    return m;
}

__device__ inline void load_rec(const GRec* __restrict__ recs, uint32_t g, GRec& e) {
    const float4* p = reinterpret_cast<const float4*>(recs + g);
    float4 a = p[0], b = p[1], c = p[2];
    e.ox = a.x; e.oy = a.y; e.ca = a.z; e.cb = a.w;
    e.cc = b.x; e.lo = b.y; e.r = b.z; e.g = b.w;
    e.b = c.x; e.x0 = __float_as_int(c.y); e.y0 = __float_as_int(c.z); e.wxy = __float_as_uint(c.w);
}

// log2(sigma G') of record e at the pixel, or -inf outside its box.
__device__ inline float rec_power(const GRec& e, int px, int py) {
    const uint32_t rx = (uint32_t)(px - e.x0), ry = (uint32_t)(py - e.y0);
    if (rx > (e.wxy & 0xffffu) || ry > (e.wxy >> 16)) return -INFINITY;
    const float dx = (float)(int)rx + e.ox, dy = (float)(int)ry + e.oy;
    return e.lo + dx * (e.ca * dx + e.cb * dy) + e.cc * dy * dy;
}

__global__ __launch_bounds__(256) void k_composite_duplex(CompositeArgs a) {
    __shared__ GRec s_rec[kBatchSlots];
    __shared__ uint8_t s_mmask[kBatchSlots];
    __shared__ uint32_t s_cmask[kBatchSlots];
    __shared__ float s_v[kBatchSlots];

    const int ntiles = a.k.TX * a.k.TY;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const PixelCoord pc = tile_pixel(tile, a.k.TX, a.k.W, a.k.H);
    const int wave = threadIdx.x >> 6;
    const uint32_t mybit = 1u << wave;
    const int tx0 = (tile % a.k.TX) * kTile, ty0 = (tile / a.k.TX) * kTile;
    const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    const int K = a.K;
    const int cells_per_batch = kBatchSlots / K < 64 ? kBatchSlots / K : 64;
    const float eps = a.o.no_et ? 0.0f : a.o.eps;

    float T = 1.0f, N0 = 0.0f, N1 = 0.0f, N2 = 0.0f, D = 0.0f;
    int32_t last = 0;
    bool done = !pc.valid;
    uint32_t nrend = 0, nval = 0;
    bool wave_done = __all(done);

    for (uint32_t b = start; b < end; b += cells_per_batch) {
        const int nb = (int)min((uint32_t)cells_per_batch, end - b);
        const int nslots = nb * K;
        __syncthreads();  // the previous batch has been consumed
        if (threadIdx.x < nb) s_cmask[threadIdx.x] = 0;
        __syncthreads();
        if (threadIdx.x < nslots) {
            const int c = threadIdx.x / K;
            const uint32_t cell = a.vals[b + c];
            GRec e;
            load_rec(a.recs, cell * K + (threadIdx.x - c * K), e);
            s_rec[threadIdx.x] = e;
            const uint32_t m = quad_mask(e, tx0, ty0);
            s_mmask[threadIdx.x] = (uint8_t)m;
            if (m) atomicOr(&s_cmask[c], m);
            if (threadIdx.x - c * K == 0) s_v[c] = a.cell_v[cell];
        }
        __syncthreads();
        if (!wave_done) {
            for (int c = 0; c < nb; c++) {
                if (!(s_cmask[c] & mybit)) continue;  // no member touches this quadrant
                if (!done && T < eps) done = true;      // cell-level early termination
                if (__all(done)) {
                    wave_done = true;
                    break;
                }
                const float v = s_v[c];
                float A0 = 0.0f, A1 = 0.0f, A2 = 0.0f, B = 0.0f, P = 1.0f;
                uint32_t cnt = 0;
                for (int kk = 0; kk < K; kk++) {
                    const int s = c * K + kk;
                    if (!(s_mmask[s] & mybit)) continue;
                    const GRec& e = s_rec[s];
                    const float pw = rec_power(e, pc.px, pc.py);
                    if (!done && pw >= a.o.log2_alpha_min) {
                        const float al = fminf(a.o.alpha_max, exp2f(pw));
                        A0 += al * e.r;
                        A1 += al * e.g;
                        A2 += al * e.b;
                        B += al;
                        P -= P * (v * al);
                        cnt++;
                    }
                }
                if (!done) {
                    const float w = v * T;
                    N0 += w * A0;
                    N1 += w * A1;
                    N2 += w * A2;
                    D += w * B;
                    T *= P;
                    if (cnt) {
                        last = (int32_t)(b + c - start + 1);
                        nrend += cnt;
                    }
                }
            }
        }
        if (a.counters) {
            // N^val: gated members of every listed cell, ignoring termination
            if (pc.valid)
                for (int s = 0; s < nslots; s++)
                    if (s_mmask[s] & mybit) nval += rec_power(s_rec[s], pc.px, pc.py) >= a.o.log2_alpha_min;
        } else if (!__syncthreads_or(!wave_done)) {
            break;
        }
    }
    if (!pc.valid) return;
    const size_t HW = (size_t)a.k.W * a.k.H, p = (size_t)pc.py * a.k.W + pc.px;
    if (D > 0.0f) {
        const float inv = 1.0f / D;
        a.color[p] = N0 * inv;
        a.color[HW + p] = N1 * inv;
        a.color[2 * HW + p] = N2 * inv;
    } else {
        a.color[p] = a.o.bg[0];
        a.color[HW + p] = a.o.bg[1];
        a.color[2 * HW + p] = a.o.bg[2];
    }
    if (a.D) a.D[p] = D;
    if (a.T) a.T[p] = T;
    if (a.last) a.last[p] = last;
    if (a.counters) {
        atomicAdd(&a.counters[0], (unsigned long long)nval);
        atomicAdd(&a.counters[1], (unsigned long long)nrend);
    }
}

__global__ __launch_bounds__(256) void k_composite_alpha(CompositeArgs a) {
    __shared__ GRec s_rec[kBatchSlots];
    __shared__ uint8_t s_mmask[kBatchSlots];

    const int ntiles = a.k.TX * a.k.TY;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const PixelCoord pc = tile_pixel(tile, a.k.TX, a.k.W, a.k.H);
    const int wave = threadIdx.x >> 6;
    const uint32_t mybit = 1u << wave;
    const int tx0 = (tile % a.k.TX) * kTile, ty0 = (tile / a.k.TX) * kTile;
    const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    const float eps = a.o.no_et ? 0.0f : a.o.eps;

    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    int32_t last = 0;
    bool done = !pc.valid;
    uint32_t nrend = 0, nval = 0;
    bool wave_done = __all(done);

    for (uint32_t b = start; b < end; b += kBatchSlots) {
        const int nb = (int)min((uint32_t)kBatchSlots, end - b);
        __syncthreads();
        if (threadIdx.x < nb) {
            GRec e;
            load_rec(a.recs, a.vals[b + threadIdx.x], e);
            s_rec[threadIdx.x] = e;
            s_mmask[threadIdx.x] = (uint8_t)quad_mask(e, tx0, ty0);
        }
        __syncthreads();
        if (!wave_done) {
            for (int s = 0; s < nb; s++) {
                if (!(s_mmask[s] & mybit)) continue;
                if (!done && T < eps) done = true;
                if (__all(done)) {
                    wave_done = true;
                    break;
                }
                const GRec& e = s_rec[s];
                const float pw = rec_power(e, pc.px, pc.py);
                if (!done && pw >= a.o.log2_alpha_min) {
                    const float al = fminf(a.o.alpha_max, exp2f(pw));
                    const float w = al * T;
                    C0 += w * e.r;
                    C1 += w * e.g;
                    C2 += w * e.b;
                    T -= w;
                    last = (int32_t)(b + s - start + 1);
                    nrend++;
                }
            }
        }
        if (a.counters) {
            if (pc.valid)
                for (int s = 0; s < nb; s++)
                    if (s_mmask[s] & mybit) nval += rec_power(s_rec[s], pc.px, pc.py) >= a.o.log2_alpha_min;
        } else if (!__syncthreads_or(!wave_done)) {
            break;
        }
    }
    if (!pc.valid) return;
    const size_t HW = (size_t)a.k.W * a.k.H, p = (size_t)pc.py * a.k.W + pc.px;
    a.color[p] = C0 + T * a.o.bg[0];
    a.color[HW + p] = C1 + T * a.o.bg[1];
    a.color[2 * HW + p] = C2 + T * a.o.bg[2];
    if (a.D) a.D[p] = 1.0f - T;
    if (a.T) a.T[p] = T;
    if (a.last) a.last[p] = last;
    if (a.counters) {
        atomicAdd(&a.counters[0], (unsigned long long)nval);
        atomicAdd(&a.counters[1], (unsigned long long)nrend);
    }
}

void launch_composite_duplex(hipStream_t st, const CompositeArgs& a) {
    const int tiles = a.k.TX * a.k.TY;
    if (tiles <= 0) return;
    hipLaunchKernelGGL(k_composite_duplex, dim3(tiles), dim3(256), 0, st, a);
}

void launch_composite_alpha(hipStream_t st, const CompositeArgs& a) {
    const int tiles = a.k.TX * a.k.TY;
    if (tiles <= 0) return;
    hipLaunchKernelGGL(k_composite_alpha, dim3(tiles), dim3(256), 0, st, a);
}

}  // namespace dgs
