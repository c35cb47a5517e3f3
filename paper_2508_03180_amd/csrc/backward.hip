// Backward pass of the hybrid renderer (Duplex mode).
//
// Forward per pixel (Sec. V-A, eq. hybrid_renderer, w_n = v_n T_n,
// eq. dulpex_T): for processed cells n,
//     A_n = sum_k a_k c_k,  B_n = sum_k a_k,  P_n = prod_k (1 - v_n a_k),
//     N = sum_n v_n T_n A_n,  D = sum_n v_n T_n B_n,  T_{n+1} = T_n P_n,
//     C = N / D.
// With g_N = dL/dC / D and g_D = -(dL/dC . C) / D + dL/dD:
//     dL/dA_n = v_n T_n g_N,  dL/dB_n = v_n T_n g_D,
//     dL/dT_n = v_n (g_N . A_n + g_D B_n) + P_n dL/dT_{n+1},
//     dL/dP_n = T_n dL/dT_{n+1},   dP_n/da_k = -v_n P_n / (1 - v_n a_k),
//     dL/dv_n = T_n (g_N . A_n + g_D B_n) - dL/dP_n sum_k a_k P_n / (1 - v_n a_k).
// The walk replays the forward's per-tile cell lists back to front from the
// replay start the forward saved (the last contributing cell whose
// transmittance in front is at least kMinReplayT, together with that
// transmittance), recovering T_n = T_{n+1} / P_n for the cells in front of
// it: there T_{n+1} >= kMinReplayT, so P_n >= kMinReplayT and the quotient
// is finite however many opaque members a cell holds.  Per-Gaussian screen-space gradients
// (mean, conic, sigma, colour) and per-cell dL/dv are reduced over each
// wavefront and added atomically; a second kernel carries them through the
// projection (EWA covariance, quaternion, scales, SH colour and its view
// direction) and a third through v_n = sigmoid(SH(d_n)).
#include "cells.h"
#include "common.h"
#include "launch.h"

namespace dgs {

constexpr int kBwdWaves = 4;
constexpr float kLog2e = 1.4426950408889634f;

// Cross-lane steps in registers (no LDS): DPP within 16-lane rows,
// v_permlane16_swap / v_permlane32_swap across rows and halves.
template <int CTRL>
__device__ inline float dpp(float v) {
    return __uint_as_float(__builtin_amdgcn_update_dpp(0u, __float_as_uint(v), CTRL, 0xf, 0xf, false));
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <- 7 - i within each 8
constexpr int kDppMirror = 0x140;     // lane i <- 15 - i within each row of 16

// x, y -> (x with its upper 32 lanes replaced by y's lower 32,
//          y with its lower 32 lanes replaced by x's upper 32); summed.
__device__ inline float swap32_sum(float x, float y) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
// x, y -> (rows 0, 2 of x with rows 0, 2 of y, rows 1, 3 of x with rows 1, 3 of y); summed.
__device__ inline float swap16_sum(float x, float y) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Wavefront total of v in every lane.
__device__ inline float wave_sum(float v) {
    v += dpp<kDppXor1>(v);
    v += dpp<kDppXor2>(v);
    v += dpp<kDppHalfMirror>(v);
    v += dpp<kDppMirror>(v);       // every lane: its row's total
    v = swap16_sum(v, v);          // rows 0+1 and 2+3
    return swap32_sum(v, v);       // all four rows
}

// Sums eight per-lane values over the wavefront with a transposed butterfly
// (each exchange step keeps half of the values and trades the other half):
// every lane of group g = lane >> 3 returns the wavefront total of value g.
__device__ inline float wave_sum8(const float (&v)[8], int lane) {
    float w4[4], w2[2];
#pragma unroll
    for (int i = 0; i < 4; i++) w4[i] = swap32_sum(v[i], v[4 + i]);    // halves: values 0..3 / 4..7
#pragma unroll
    for (int i = 0; i < 2; i++) w2[i] = swap16_sum(w4[i], w4[2 + i]);  // row r: values 2r, 2r + 1
    const bool b3 = (lane & 8) != 0;
    float w = (b3 ? w2[1] : w2[0]) + dpp<kDppMirror>(b3 ? w2[0] : w2[1]);  // half h of row r: value 2r + h
    w += dpp<kDppHalfMirror>(w);
    w += dpp<kDppXor1>(w);
    w += dpp<kDppXor2>(w);
    return w;
}

struct BRec {
    float ox, oy, ca, cb, cc, lo;  // as stored: log2(sigma G') = lo + ca dx^2 + cb dx dy + cc dy^2
    float A, B, C, sigma, r, g, b;  // natural-domain conic and sigma, for the gradients
    int x0, y0;
    uint32_t wx, wy;
};

// lo + ca dx^2 + cb dx dy + cc dy^2 in the forward compositor's operations.
// With lo = log2 sigma + log2 v (the forward's staged record) this is the
// forward's gate power log2(v sigma G'), reproduced bit for bit with its
// alpha_min threshold log2 alpha_min + log2 v, so every gate decision (box,
// alpha_min) is the forward's; minus log2 v it is log2(sigma G') for the
// gradients (continuous: the extra rounding does not matter there).
// Outside the box's columns (inx false) the power is -inf, which the
// alpha_min test rejects as the forward's box test does.
__device__ inline float brec_power(const BRec& e, float lo, float dx, float dy, bool inx) {
    const float t0 = inx ? fmaf(e.ca * dx, dx, lo) : -INFINITY;
    const float t1 = e.cb * dx;
    return fmaf(dy, fmaf(e.cc, dy, t1), t0);
}

typedef float F4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) const F4 LdsF4;

// The wavefront's record array as a 32-bit LDS address in a scalar register
// (every lane reads the same record).
__device__ inline uint32_t lds_base(const GRec* lds) {
    return __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(const LdsF4*)lds);
}

__device__ inline BRec read_brec(uint32_t lb, int i) {
    const LdsF4* p = (const LdsF4*)(uintptr_t)(lb + (uint32_t)i * (uint32_t)sizeof(GRec));
    const F4 a = p[0], b = p[1], c = p[2];
    BRec e;
    e.ox = a.x; e.oy = a.y;
    e.ca = a.z; e.cb = a.w; e.cc = b.x;
    // stored log2-domain coefficients -> conic of the dilated covariance
    e.A = a.z * (-2.0f / kLog2e);
    e.B = a.w * (-1.0f / kLog2e);
    e.C = b.x * (-2.0f / kLog2e);
    e.lo = b.y;
    e.sigma = __builtin_amdgcn_exp2f(b.y);
    e.r = b.z; e.g = b.w; e.b = c.x;
    e.x0 = __float_as_int(c.y);
    e.y0 = __float_as_int(c.z);
    const uint32_t wxy = __float_as_uint(c.w);
    e.wx = wxy & 0xffffu;
    e.wy = wxy >> 16;
    return e;
}

// Backward of a whole 16x16 tile (NS = 4: lane l holds pixel (l & 15,
// 4 j + (l >> 4)) of strip j) or of one 16x8 half (NS = 2, strips s0 and
// s0 + 1), in the forward compositor's layout and with its exact gate
// arithmetic.  Each
// pixel walks back from its own last contributing entry; per member, the
// lane first sums its pixels' contributions, then the wavefront reduces
// them once for the tile.
template <int NS, bool RAGGED>
__device__ inline void duplex_tile_bwd(const BwdArgs& a, int tile, int s0, int lane, GRec* lds) {
    const CamK& k = a.k;
    const int tx0 = (tile % k.TX) * kTile, ty0 = (tile / k.TX) * kTile;
    const int px = tx0 + (lane & 15), py0 = ty0 + 4 * s0 + (lane >> 4);
    const uint32_t start = a.ranges[2 * tile], len = a.ranges[2 * tile + 1] - start;
    const int K = a.K;
    const uint32_t kmask = member_mask(K);
    const float th = a.o.log2_alpha_min, amax = a.o.alpha_max;
    const size_t HW = (size_t)k.W * k.H;
    const uint32_t lb = lds_base(lds);

    int32_t last[NS];
    float gN0[NS], gN1[NS], gN2[NS], gD[NS], T[NS], R[NS];
    int maxlast = 0;
#pragma unroll
    for (int j = 0; j < NS; j++) {
        const int py = py0 + 4 * j;
        last[j] = 0;
        gN0[j] = gN1[j] = gN2[j] = gD[j] = 0.0f;
        T[j] = 1.0f;
        R[j] = 0.0f;  // dL/dT after the current cell
        if (px < k.W && py < k.H) {
            const size_t pi = (size_t)py * k.W + px;
            const int32_t l = min(a.last[pi], (int32_t)len);  // never walk past this tile's list
            const float D = a.D[pi];
            if (D > 0.0f && l > 0) {
                const float invD = 1.0f / D;
                const float g0 = a.grad_color[pi], g1 = a.grad_color[HW + pi], g2 = a.grad_color[2 * HW + pi];
                gN0[j] = g0 * invD; gN1[j] = g1 * invD; gN2[j] = g2 * invD;
                gD[j] = -(g0 * a.color[pi] + g1 * a.color[HW + pi] + g2 * a.color[2 * HW + pi]) * invD;
                if (a.grad_D) gD[j] += a.grad_D[pi];
                T[j] = a.T[pi];  // transmittance in front of the replay start
                last[j] = l;
            }
        }
        maxlast = max(maxlast, last[j]);
    }
    // the wave walks from its largest `last` down to the first cell
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) maxlast = max(maxlast, __shfl_xor(maxlast, o, 64));
    maxlast = __builtin_amdgcn_readfirstlane(maxlast);  // uniform: scalar loop control
    for (int hi = maxlast; hi > 0;) {
        // chunk of whole cells [lo_c, hi) (list positions relative to start)
        const int nch = cells_fitting_back<RAGGED>(a.vals, a.offs, K, start, start + (uint32_t)hi, lane);
        const int lo_c = hi - nch;
        CellChunk ch;
        load_cells<RAGGED>(a.vals, a.offs, a.cell_v, K, start + (uint32_t)lo_c, start + (uint32_t)hi, nch, lane, ch);
        uint32_t sm = 0, rcols = 0;  // strips and tile columns this lane's record touches
        if (ch.g >= 0) {
            const float4* p = reinterpret_cast<const float4*>(a.recs + ch.g);
            float4* d = reinterpret_cast<float4*>(lds + lane);
            const float4 r0 = p[0], r1 = p[1], r2 = p[2];
            d[0] = r0; d[1] = r1; d[2] = r2;
            const int x0 = __float_as_int(r2.y), y0 = __float_as_int(r2.z);
            const uint32_t wxy = __float_as_uint(r2.w);
            const int x1 = x0 + (int)(wxy & 0xffffu), y1 = y0 + (int)(wxy >> 16);
            if (x0 <= tx0 + 15 && x1 >= tx0) {
                const int lo = max(x0, tx0) - tx0, hi = min(x1, tx0 + 15) - tx0;
                rcols = ((2u << (hi - lo)) - 1u) << lo;
#pragma unroll
                for (int j = 0; j < NS; j++) {
                    const int sy0 = ty0 + 4 * (s0 + j);
                    if (y0 <= sy0 + 3 && y1 >= sy0) sm |= 1u << j;
                }
            }
        }
        uint64_t Bm[NS];
#pragma unroll
        for (int j = 0; j < NS; j++) Bm[j] = __ballot((sm >> j) & 1u);
        for (int c = nch - 1; c >= 0; c--) {
            // fixed K: cell c holds record lanes cK .. cK + K - 1
            const int base = RAGGED ? lane_value(ch.first, c) : c * K;
            const uint32_t cm = RAGGED ? member_mask(lane_value(ch.cnt, c)) : kmask;
            const int p = lo_c + c;  // list position (0-based) of this cell
            uint32_t mj[NS], mm = 0;
            bool act[NS];
            uint64_t am[NS], amall = 0;  // ballots of act (ballots of single compares)
            float thj[NS];  // gate threshold, +inf where the pixel does not reach this cell
            const float v = __int_as_float(lane_value(__float_as_int(ch.vc), c));
            const float lv = fold_log2_weight(v);  // as the forward stages it
            const float thc = th + lv;
#pragma unroll
            for (int j = 0; j < NS; j++) {
                mj[j] = (uint32_t)(Bm[j] >> base) & cm;
                mm |= mj[j];
                act[j] = p < last[j];
                thj[j] = act[j] ? thc : INFINITY;
                am[j] = __ballot(p < last[j]);
                amall |= am[j];
            }
            if (!mm || !amall) continue;  // no member touches the owned rows / no pixel reaches the cell
            {
                // drop the members whose box misses every pixel that reaches
                // this cell: they change nothing there (the other pixels have
                // threshold +inf), so the cell's replay is the same without them
                uint32_t live = 0;
#pragma unroll
                for (int j = 0; j < NS; j++) {
                    if (am[j] != ~0ull) {
                        uint32_t ac = (uint32_t)(am[j] | (am[j] >> 32));
                        ac = (ac | (ac >> 16)) & 0xffffu;  // columns (lane & 15) with a pixel reaching the cell
                        // Bm[j]: the records touching strip j
                        mj[j] = (uint32_t)((__ballot((rcols & ac) != 0u) & Bm[j]) >> base) & cm;
                    }
                    live |= mj[j];
                }
                mm = live;
                if (!mm) continue;
            }
            const uint32_t cell = (uint32_t)lane_value((int)ch.id, c);
            const int gfirst = lane_value(ch.gfirst, c);  // Gaussian of member 0
            // pass 1: cell totals at each pixel (same decisions as the forward)
            float A0[NS], A1[NS], A2[NS], Bs[NS], P[NS];
#pragma unroll
            for (int j = 0; j < NS; j++) { A0[j] = A1[j] = A2[j] = Bs[j] = 0.0f; P[j] = 1.0f; }
            for (uint32_t rem = mm; rem; rem &= rem - 1) {
                const int kk = __builtin_ctz(rem);
                const BRec e = read_brec(lb, base + kk);
                const uint32_t rx = (uint32_t)(px - e.x0);
                const bool inx = rx <= e.wx;
                const float dx = (float)(int)rx + e.ox;
                const float lof = e.lo + lv;
                const uint32_t ry0 = (uint32_t)(py0 - e.y0);
                const float dy0 = (float)(int)ry0 + e.oy;
#pragma unroll
                for (int j = 0; j < NS; j++) {
                    const uint32_t ry = ry0 + 4u * j;
                    const float dy = j ? dy0 + 4.0f * j : dy0;  // as the forward forms it
                    const float pwv = brec_power(e, lof, dx, dy, inx);  // log2(v sigma G')
                    if ((ry <= e.wy) & (pwv >= thj[j])) {
                        const float al = fminf(amax, __builtin_amdgcn_exp2f(pwv - lv));
                        A0[j] = fmaf(al, e.r, A0[j]); A1[j] = fmaf(al, e.g, A1[j]); A2[j] = fmaf(al, e.b, A2[j]);
                        Bs[j] += al;
                        P[j] = fmaf(-P[j], v * al, P[j]);
                    }
                }
            }
            float dLdA0[NS], dLdA1[NS], dLdA2[NS], dLdB[NS], dLdP[NS];
            float dv = 0.0f;
#pragma unroll
            for (int j = 0; j < NS; j++) {
                dLdA0[j] = dLdA1[j] = dLdA2[j] = dLdB[j] = dLdP[j] = 0.0f;
                if (act[j]) {
                    // transmittance in front of this cell: stored for the replay
                    // start, else recovered from the one behind it (gradients
                    // are continuous: the hardware reciprocal, not a correctly
                    // rounded division)
                    const float Tn = p == last[j] - 1 ? T[j] : T[j] * __builtin_amdgcn_rcpf(P[j]);
                    const float w = v * Tn;
                    dLdA0[j] = w * gN0[j]; dLdA1[j] = w * gN1[j]; dLdA2[j] = w * gN2[j];
                    dLdB[j] = w * gD[j];
                    const float dLdw = gN0[j] * A0[j] + gN1[j] * A1[j] + gN2[j] * A2[j] + gD[j] * Bs[j];
                    dLdP[j] = Tn * R[j];
                    dv += Tn * dLdw;
                    R[j] = v * dLdw + P[j] * R[j];
                    T[j] = Tn;
                }
            }
            // pass 2: per-member gradients, summed over the lane's pixels, then the wave
            for (uint32_t rem = mm; rem; rem &= rem - 1) {
                const int kk = __builtin_ctz(rem);
                const BRec e = read_brec(lb, base + kk);
                const uint32_t rx = (uint32_t)(px - e.x0);
                const bool inx = rx <= e.wx;
                const float dx = (float)(int)rx + e.ox;
                const float lof = e.lo + lv;
                const uint32_t ry0 = (uint32_t)(py0 - e.y0);
                const float dy0 = (float)(int)ry0 + e.oy;
                // dL/dp per pixel (gp) enters the mean, conic and sigma
                // gradients only through gp, gp dy and gp dy^2 (dx is the
                // lane's constant for this member), so the lane sums those
                // three and forms the seven quantities once per member
                float S0 = 0.f, S1 = 0.f, S2 = 0.f, gr = 0.f, gg = 0.f, gb = 0.f;
                bool anyhit = false;
#pragma unroll
                for (int j = 0; j < NS; j++) {
                    const uint32_t ry = ry0 + 4u * j;
                    const float dy = j ? dy0 + 4.0f * j : dy0;
                    const float pwv = brec_power(e, lof, dx, dy, inx);
                    if ((ry <= e.wy) & (pwv >= thj[j])) {
                        anyhit = true;
                        const float sg = __builtin_amdgcn_exp2f(pwv - lv);  // sigma G'
                        const float al = fminf(amax, sg);
                        const float om = 1.0f - v * al;
                        const float Pom = dLdP[j] * P[j] * __builtin_amdgcn_rcpf(om);  // dL/dP * P / (1 - v al)
                        dv -= Pom * al;
                        const float dLda = dLdA0[j] * e.r + dLdA1[j] * e.g + dLdA2[j] * e.b + dLdB[j] - Pom * v;
                        gr += dLdA0[j] * al; gg += dLdA1[j] * al; gb += dLdA2[j] * al;
                        // alpha = sigma exp(p) below the clamp: dalpha/dp = alpha
                        const float gp = sg < amax ? dLda * al : 0.0f;
                        S0 += gp;
                        S1 = fmaf(gp, dy, S1);
                        S2 = fmaf(gp * dy, dy, S2);
                    }
                }
                // p = lo + ca dx^2 + cb dx dy + cc dy^2 with dx = px + 0.5 - u
                // (and dy likewise): dp/du = (A dx + B dy, B dx + C dy) for
                // the natural conic (A, B, C); dp/dA = -dx^2/2, dp/dB = -dx dy,
                // dp/dC = -dy^2/2; dalpha/dsigma = alpha / sigma
                const float gu0 = e.A * dx * S0 + e.B * S1, gu1 = e.B * dx * S0 + e.C * S1;
                const float gA = -0.5f * dx * dx * S0, gB = -dx * S1, gC = -0.5f * S2;
                const float gs = S0 * __builtin_amdgcn_rcpf(e.sigma);
                if (__any(anyhit)) {
                    // quantities 0..7 by one transposed reduction (group q of
                    // eight lanes holds quantity q), quantity 8 by a plain one;
                    // one atomic instruction, nine lanes, one 64-byte row
                    const float s8[8] = {gu0, gu1, gA, gB, gC, gs, gr, gg};
                    const float t8 = wave_sum8(s8, lane);
                    const float tb = wave_sum(gb);
                    const bool head = (lane & 7) == 0;
                    const float t = head ? t8 : tb;
                    const int q = head ? (lane >> 3) : 8;
                    if ((head || lane == 1) && t != 0.0f)
                        atomicAdd(&a.g2d[((size_t)gfirst + kk) * kG2dRow + q], t);
                }
            }
            const float dvs = wave_sum(dv);
            if (lane == 0 && dvs != 0.0f) atomicAdd(&a.gv[cell], dvs);
        }
        hi = lo_c;
    }
}

template <bool RAGGED>
__global__ __launch_bounds__(256) void k_composite_bwd(BwdArgs a) {
    __shared__ GRec s_rec[kBwdWaves][64];
    a.k = a.fr->k;
    a.o = a.fr->o;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    GRec* lds = s_rec[wave];
    const uint32_t nitems = a.queue[1];
    for (;;) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(a.queue, 1u);
        // lane 0's ticket in a scalar register: the item, its tile and its
        // half are then wavefront-uniform, and so is all loop control below
        t = __builtin_amdgcn_readfirstlane(t);
        if (t >= nitems) break;
        const uint32_t item = a.order[t];
        const int tile = (int)(item >> 3), mode = (int)(item & 7u);
        // half-tile items (the tiles with the longest lists, which set the
        // kernel's span) issue ahead of whole-tile items on their SIMD
        if (mode != 0)
            __builtin_amdgcn_s_setprio(3);
        else
            __builtin_amdgcn_s_setprio(0);
        if (mode == 0)
            duplex_tile_bwd<4, RAGGED>(a, tile, 0, lane, lds);
        else
            duplex_tile_bwd<2, RAGGED>(a, tile, 2 * (mode - 2), lane, lds);
    }
}

// ---------------------------------------------------------------- projection

// Real SH basis (as in the forward) and its gradient in the direction.
__device__ inline void sh_basis_grad(int deg, float x, float y, float z, float* Y, float* gx, float* gy,
                                     float* gz) {
    const float c0 = 0.28209479177387814f, c1 = 0.4886025119029199f;
    Y[0] = c0; gx[0] = gy[0] = gz[0] = 0.f;
    if (deg < 1) return;
    Y[1] = -c1 * y; gx[1] = 0.f; gy[1] = -c1; gz[1] = 0.f;
    Y[2] = c1 * z;  gx[2] = 0.f; gy[2] = 0.f; gz[2] = c1;
    Y[3] = -c1 * x; gx[3] = -c1; gy[3] = 0.f; gz[3] = 0.f;
    if (deg < 2) return;
    const float k4 = 1.0925484305920792f, k6 = 0.31539156525252005f, k8 = 0.5462742152960396f;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = k4 * x * y;                gx[4] = k4 * y;          gy[4] = k4 * x;           gz[4] = 0.f;
    Y[5] = -k4 * y * z;               gx[5] = 0.f;             gy[5] = -k4 * z;          gz[5] = -k4 * y;
    Y[6] = k6 * (2.f * zz - xx - yy); gx[6] = -2.f * k6 * x;   gy[6] = -2.f * k6 * y;    gz[6] = 4.f * k6 * z;
    Y[7] = -k4 * x * z;               gx[7] = -k4 * z;         gy[7] = 0.f;              gz[7] = -k4 * x;
    Y[8] = k8 * (xx - yy);            gx[8] = 2.f * k8 * x;    gy[8] = -2.f * k8 * y;    gz[8] = 0.f;
    if (deg < 3) return;
    const float k9 = 0.5900435899266435f, k10 = 2.890611442640554f, k11 = 0.4570457994644658f;
    const float k12 = 0.3731763325901154f, k14 = 1.445305721320277f;
    Y[9] = -k9 * y * (3.f * xx - yy);
    gx[9] = -6.f * k9 * x * y; gy[9] = -k9 * (3.f * xx - 3.f * yy); gz[9] = 0.f;
    Y[10] = k10 * x * y * z;
    gx[10] = k10 * y * z; gy[10] = k10 * x * z; gz[10] = k10 * x * y;
    Y[11] = -k11 * y * (4.f * zz - xx - yy);
    gx[11] = 2.f * k11 * x * y; gy[11] = -k11 * (4.f * zz - xx - 3.f * yy); gz[11] = -8.f * k11 * y * z;
    Y[12] = k12 * z * (2.f * zz - 3.f * xx - 3.f * yy);
    gx[12] = -6.f * k12 * x * z; gy[12] = -6.f * k12 * y * z; gz[12] = k12 * (6.f * zz - 3.f * xx - 3.f * yy);
    Y[13] = -k11 * x * (4.f * zz - xx - yy);
    gx[13] = -k11 * (4.f * zz - 3.f * xx - yy); gy[13] = 2.f * k11 * x * y; gz[13] = -8.f * k11 * x * z;
    Y[14] = k14 * z * (xx - yy);
    gx[14] = 2.f * k14 * x * z; gy[14] = -2.f * k14 * y * z; gz[14] = k14 * (xx - yy);
    Y[15] = -k9 * x * (xx - 3.f * yy);
    gx[15] = -k9 * (3.f * xx - 3.f * yy); gy[15] = 6.f * k9 * x * y; gz[15] = 0.f;
}

// Adds the gradient g (w.r.t. the unit direction d = (p - o)/|p - o|) to the
// gradient of p: (I - d d^T) g / |p - o|.
__device__ inline void dir_to_pos(const float* d, float len, const float* g, float* gp) {
    const float dg = d[0] * g[0] + d[1] * g[1] + d[2] * g[2];
    for (int i = 0; i < 3; i++) gp[i] += (g[i] - d[i] * dg) / len;
}

// dst = v (OW: the caller's buffer is written, not read) or dst += v.
template <bool OW>
__device__ inline void put(float* dst, float v) {
    if constexpr (OW) *dst = v;
    else *dst += v;
}

// DEG: the scene's SH degree (0..3) as a constant, so that every loop over
// the coefficients unrolls and their loads issue together.
template <bool OW, int DEG>
__global__ __launch_bounds__(256) void k_gauss_project_bwd(BwdArgs a, ProjBwdArgs b) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.M) return;
    a.k = a.fr->k;
    a.o = a.fr->o;
    const int M = a.M;
    const float4* row = reinterpret_cast<const float4*>(a.g2d + (size_t)g * kG2dRow);
    const float4 r0 = row[0], r1 = row[1];
    const float s9[9] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w, a.g2d[(size_t)g * kG2dRow + 8]};
    bool any = false;
#pragma unroll
    for (int i = 0; i < 9; i++) any = any || s9[i] != 0.0f;
    if (!any) {
        if constexpr (OW) {  // no gradient reaches this Gaussian: its entries are zero
            for (int i = 0; i < 3; i++) b.d_means[(size_t)i * M + g] = b.d_scales[(size_t)i * M + g] = 0.0f;
            for (int i = 0; i < 4; i++) b.d_rots[(size_t)i * M + g] = 0.0f;
            b.d_opac[g] = 0.0f;
            constexpr int C3 = 3 * (DEG + 1) * (DEG + 1);
#pragma unroll
            for (int i = 0; i < C3; i++) b.d_sh[(size_t)i * M + g] = 0.0f;
            if (b.d_mean2d) b.d_mean2d[g] = b.d_mean2d[M + g] = 0.0f;
        }
        return;
    }
    const CamK& k = a.k;
    const float m0 = b.means[g], m1 = b.means[M + g], m2 = b.means[2 * M + g];
    float t[3];
    for (int i = 0; i < 3; i++) t[i] = k.R[3 * i] * m0 + k.R[3 * i + 1] * m1 + k.R[3 * i + 2] * m2 + k.t[i];
    const float tz = t[2], itz = 1.0f / tz;
    // rotation from the normalised quaternion
    const float q0 = b.rots[g], q1 = b.rots[M + g], q2 = b.rots[2 * M + g], q3 = b.rots[3 * M + g];
    const float qn = sqrtf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    const float w = q0 / qn, x = q1 / qn, y = q2 / qn, z = q3 / qn;
    float R[9];
    R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z);       R[2] = 2.f * (x * z + w * y);
    R[3] = 2.f * (x * y + w * z);       R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
    R[6] = 2.f * (x * z - w * y);       R[7] = 2.f * (y * z + w * x);       R[8] = 1.f - 2.f * (x * x + y * y);
    const float s[3] = {b.scales[g], b.scales[M + g], b.scales[2 * M + g]};
    float Mq[9], Sig[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) Mq[3 * i + j] = R[3 * i + j] * s[j];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            Sig[3 * i + j] = Mq[3 * i] * Mq[3 * j] + Mq[3 * i + 1] * Mq[3 * j + 1] + Mq[3 * i + 2] * Mq[3 * j + 2];
    // Jacobian of the perspective map, with the frustum clamp
    const float limx = 1.3f * (0.5f * k.W / k.fx), limy = 1.3f * (0.5f * k.H / k.fy);
    const float rx = t[0] * itz, ry = t[1] * itz;
    const bool cx_in = rx > -limx && rx < limx, cy_in = ry > -limy && ry < limy;
    const float xr = fminf(limx, fmaxf(-limx, rx)), yr = fminf(limy, fmaxf(-limy, ry));
    const float J00 = k.fx * itz, J02 = -k.fx * xr * itz, J11 = k.fy * itz, J12 = -k.fy * yr * itz;
    float Mx[6];  // J W, 2 x 3
    for (int j = 0; j < 3; j++) {
        Mx[j] = J00 * k.R[j] + J02 * k.R[6 + j];
        Mx[3 + j] = J11 * k.R[3 + j] + J12 * k.R[6 + j];
    }
    float cov[3];  // xx, xy, yy of M Sigma M^T (plus dilation below)
    {
        float MS[6];
        for (int r = 0; r < 2; r++)
            for (int j = 0; j < 3; j++)
                MS[3 * r + j] = Mx[3 * r] * Sig[j] + Mx[3 * r + 1] * Sig[3 + j] + Mx[3 * r + 2] * Sig[6 + j];
        cov[0] = MS[0] * Mx[0] + MS[1] * Mx[1] + MS[2] * Mx[2];
        cov[1] = MS[0] * Mx[3] + MS[1] * Mx[4] + MS[2] * Mx[5];
        cov[2] = MS[3] * Mx[3] + MS[4] * Mx[4] + MS[5] * Mx[5];
    }
    const float a_ = cov[0] + a.o.delta, b_ = cov[1], c_ = cov[2] + a.o.delta;
    const float det = a_ * c_ - b_ * b_;
    const float QA = c_ / det, QB = -b_ / det, QC = a_ / det;
    // conic gradient -> covariance gradient: dL/dS = -Q Gq Q (Gq symmetric, off-diagonal gB/2)
    const float gA = s9[2], gBh = 0.5f * s9[3], gC = s9[4];
    const float t00 = QA * gA + QB * gBh, t01 = QA * gBh + QB * gC;
    const float t10 = QB * gA + QC * gBh, t11 = QB * gBh + QC * gC;
    const float dS00 = -(t00 * QA + t01 * QB), dS01 = -(t00 * QB + t01 * QC), dS11 = -(t10 * QB + t11 * QC);
    // Sigma' = Mx Sigma Mx^T: dL/dMx = 2 G Mx Sigma, dL/dSigma = Mx^T G Mx (G per-entry symmetric)
    const float G2[4] = {dS00, dS01, dS01, dS11};
    float MSig[6];
    for (int r = 0; r < 2; r++)
        for (int j = 0; j < 3; j++)
            MSig[3 * r + j] = Mx[3 * r] * Sig[j] + Mx[3 * r + 1] * Sig[3 + j] + Mx[3 * r + 2] * Sig[6 + j];
    float gMx[6];
    for (int r = 0; r < 2; r++)
        for (int j = 0; j < 3; j++) gMx[3 * r + j] = 2.f * (G2[2 * r] * MSig[j] + G2[2 * r + 1] * MSig[3 + j]);
    float gSig[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            gSig[3 * i + j] = Mx[i] * (G2[0] * Mx[j] + G2[1] * Mx[3 + j]) + Mx[3 + i] * (G2[2] * Mx[j] + G2[3] * Mx[3 + j]);
    // Sigma = Mq Mq^T: dL/dMq = 2 gSig Mq
    float gMq[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            gMq[3 * i + j] = 2.f * (gSig[3 * i] * Mq[j] + gSig[3 * i + 1] * Mq[3 + j] + gSig[3 * i + 2] * Mq[6 + j]);
    float gs[3] = {0.f, 0.f, 0.f}, gR[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            gs[j] += gMq[3 * i + j] * R[3 * i + j];
            gR[3 * i + j] = gMq[3 * i + j] * s[j];
        }
    // rotation -> normalised quaternion -> quaternion
    const float gw = 2.f * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
    const float gx = 2.f * (y * gR[1] + z * gR[2] + y * gR[3] - 2.f * x * gR[4] - w * gR[5] + z * gR[6] +
                            w * gR[7] - 2.f * x * gR[8]);
    const float gy = 2.f * (-2.f * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] +
                            z * gR[7] - 2.f * y * gR[8]);
    const float gz = 2.f * (-2.f * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.f * z * gR[4] + y * gR[5] +
                            x * gR[6] + y * gR[7]);
    const float qd = w * gw + x * gx + y * gy + z * gz;
    put<OW>(&b.d_rots[g], (gw - w * qd) / qn);
    put<OW>(&b.d_rots[M + g], (gx - x * qd) / qn);
    put<OW>(&b.d_rots[2 * M + g], (gy - y * qd) / qn);
    put<OW>(&b.d_rots[3 * M + g], (gz - z * qd) / qn);
    for (int j = 0; j < 3; j++) put<OW>(&b.d_scales[(size_t)j * M + g], gs[j]);
    // Mx = J W: dL/dJ = dL/dMx W^T, then J (and the mean u) -> camera-space position
    const float gJ00 = gMx[0] * k.R[0] + gMx[1] * k.R[1] + gMx[2] * k.R[2];
    const float gJ02 = gMx[0] * k.R[6] + gMx[1] * k.R[7] + gMx[2] * k.R[8];
    const float gJ11 = gMx[3] * k.R[3] + gMx[4] * k.R[4] + gMx[5] * k.R[5];
    const float gJ12 = gMx[3] * k.R[6] + gMx[4] * k.R[7] + gMx[5] * k.R[8];
    const float itz2 = itz * itz;
    float gt[3];
    const float gu0 = s9[0], gu1 = s9[1];
    // u = f t_xy / t_z + c
    gt[0] = gu0 * k.fx * itz;
    gt[1] = gu1 * k.fy * itz;
    gt[2] = -(gu0 * k.fx * t[0] + gu1 * k.fy * t[1]) * itz2;
    // J00 = fx / tz, J11 = fy / tz
    gt[2] += -(gJ00 * k.fx + gJ11 * k.fy) * itz2;
    // J02 = -fx xr / tz with xr = t_x / t_z inside the clamp
    gt[2] += gJ02 * k.fx * xr * itz2 + gJ12 * k.fy * yr * itz2;
    if (cx_in) {
        gt[0] += gJ02 * (-k.fx * itz) * itz;
        gt[2] += gJ02 * (-k.fx * itz) * (-t[0] * itz2);
    }
    if (cy_in) {
        gt[1] += gJ12 * (-k.fy * itz) * itz;
        gt[2] += gJ12 * (-k.fy * itz) * (-t[1] * itz2);
    }
    float gm[3];
    for (int j = 0; j < 3; j++) gm[j] = k.R[j] * gt[0] + k.R[3 + j] * gt[1] + k.R[6 + j] * gt[2];
    // colour: c = max(0, 0.5 + sum sh Y(d)), d = (mu - o) / |mu - o|
    float dd[3] = {m0 - k.o[0], m1 - k.o[1], m2 - k.o[2]};
    const float len = sqrtf(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
    for (int i = 0; i < 3; i++) dd[i] /= len;
    constexpr int Cn = (DEG + 1) * (DEG + 1);
    float Y[16], Yx[16], Yy[16], Yz[16];
    sh_basis_grad(DEG, dd[0], dd[1], dd[2], Y, Yx, Yy, Yz);
    float gdir[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int ch = 0; ch < 3; ch++) {
        const float gc = s9[6 + ch];
        float c[Cn];
        float cval = 0.5f;
#pragma unroll
        for (int j = 0; j < Cn; j++) {
            c[j] = b.sh[((size_t)j * 3 + ch) * M + g];
            cval += Y[j] * c[j];
        }
        if (gc == 0.0f || cval < 0.0f) {  // no gradient, or a clamped colour channel
            if constexpr (OW) {
#pragma unroll
                for (int j = 0; j < Cn; j++) b.d_sh[((size_t)j * 3 + ch) * M + g] = 0.0f;
            }
            continue;
        }
#pragma unroll
        for (int j = 0; j < Cn; j++) {
            put<OW>(&b.d_sh[((size_t)j * 3 + ch) * M + g], gc * Y[j]);
            gdir[0] += gc * c[j] * Yx[j];
            gdir[1] += gc * c[j] * Yy[j];
            gdir[2] += gc * c[j] * Yz[j];
        }
    }
    dir_to_pos(dd, len, gdir, gm);
    for (int j = 0; j < 3; j++) put<OW>(&b.d_means[(size_t)j * M + g], gm[j]);
    put<OW>(&b.d_opac[g], s9[5]);
    if (b.d_mean2d) {
        put<OW>(&b.d_mean2d[g], gu0);
        put<OW>(&b.d_mean2d[M + g], gu1);
    }
}

template <bool OW, int VDEG>
__global__ __launch_bounds__(256) void k_cell_bwd(BwdArgs a, ProjBwdArgs b) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= b.N) return;
    a.k = a.fr->k;
    a.o = a.fr->o;
    const float gv = a.o.v_one ? 0.0f : a.gv[n];  // v = 1: v's parameters have no gradient
    if (gv == 0.0f) {
        if constexpr (OW) {
            constexpr int Cv = (VDEG + 1) * (VDEG + 1);
#pragma unroll
            for (int j = 0; j < Cv; j++) b.d_cell_v_sh[(size_t)j * b.N + n] = 0.0f;
            for (int j = 0; j < 3; j++) b.d_cell_pos[(size_t)j * b.N + n] = 0.0f;
        }
        return;
    }
    const CamK& k = a.k;
    const int N = b.N;
    const float p0 = b.cell_pos[n], p1 = b.cell_pos[N + n], p2 = b.cell_pos[2 * N + n];
    float dd[3] = {p0 - k.o[0], p1 - k.o[1], p2 - k.o[2]};
    const float len = sqrtf(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
    for (int i = 0; i < 3; i++) dd[i] /= len;
    constexpr int Cn = (VDEG + 1) * (VDEG + 1);
    float Y[16], Yx[16], Yy[16], Yz[16];
    sh_basis_grad(VDEG, dd[0], dd[1], dd[2], Y, Yx, Yy, Yz);
    float c[Cn], sv = 0.f;
#pragma unroll
    for (int j = 0; j < Cn; j++) {
        c[j] = b.cell_v_sh[(size_t)j * N + n];
        sv += Y[j] * c[j];
    }
    const float v = 1.0f / (1.0f + __expf(-sv));
    const float gs = gv * v * (1.0f - v);
    float gdir[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < Cn; j++) {
        put<OW>(&b.d_cell_v_sh[(size_t)j * N + n], gs * Y[j]);
        gdir[0] += gs * c[j] * Yx[j];
        gdir[1] += gs * c[j] * Yy[j];
        gdir[2] += gs * c[j] * Yz[j];
    }
    float gp[3] = {0.f, 0.f, 0.f};
    dir_to_pos(dd, len, gdir, gp);
    for (int j = 0; j < 3; j++) put<OW>(&b.d_cell_pos[(size_t)j * N + n], gp[j]);
}

void launch_composite_bwd(hipStream_t st, const BwdArgs& a) {
    const int tiles = a.k.TX * a.k.TY;
    if (tiles <= 0) return;
    const int waves = 4 * tiles < 256 * 4 * 4 ? 4 * tiles : 256 * 4 * 4;
    const dim3 g((waves + kBwdWaves - 1) / kBwdWaves), b(256);
    if (a.offs)
        hipLaunchKernelGGL(k_composite_bwd<true>, g, b, 0, st, a);
    else
        hipLaunchKernelGGL(k_composite_bwd<false>, g, b, 0, st, a);
}

template <bool OW, int DEG>
static void gauss_bwd(hipStream_t st, const BwdArgs& a, const ProjBwdArgs& b) {
    hipLaunchKernelGGL((k_gauss_project_bwd<OW, DEG>), dim3((a.M + 255) / 256), dim3(256), 0, st, a, b);
}

template <bool OW, int VDEG>
static void cell_bwd(hipStream_t st, const BwdArgs& a, const ProjBwdArgs& b) {
    hipLaunchKernelGGL((k_cell_bwd<OW, VDEG>), dim3((b.N + 255) / 256), dim3(256), 0, st, a, b);
}

// Degrees were checked against 0..3 when the frame was rendered.
template <bool OW>
static void project_bwd(hipStream_t st, const BwdArgs& a, const ProjBwdArgs& b) {
    if (a.M > 0) {
        switch (b.sh_degree) {
            case 0: gauss_bwd<OW, 0>(st, a, b); break;
            case 1: gauss_bwd<OW, 1>(st, a, b); break;
            case 2: gauss_bwd<OW, 2>(st, a, b); break;
            default: gauss_bwd<OW, 3>(st, a, b);
        }
    }
    if (b.N > 0) {
        switch (b.v_sh_degree) {
            case 0: cell_bwd<OW, 0>(st, a, b); break;
            case 1: cell_bwd<OW, 1>(st, a, b); break;
            case 2: cell_bwd<OW, 2>(st, a, b); break;
            default: cell_bwd<OW, 3>(st, a, b);
        }
    }
}

void launch_project_bwd(hipStream_t st, const BwdArgs& a, const ProjBwdArgs& b) {
    if (b.overwrite) project_bwd<true>(st, a, b);
    else project_bwd<false>(st, a, b);
}

}  // namespace dgs
