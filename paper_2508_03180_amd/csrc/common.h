// Internal definitions shared by the HIP kernels and the C-ABI host code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dgs {

constexpr int kTile = 16;        // screen tile edge, pixels
constexpr int kMaxK = 32;        // Gaussians per cell supported by the compositor
constexpr int kBatchSlots = 256; // Gaussian records staged in LDS per batch
constexpr int kXcds = 8;         // MI355X: 8 accelerator complex dies
constexpr int kMaxFeature = 64;  // neural decode: latent feature size limit
constexpr int kMaxHidden = 64;   // neural decode: hidden layer size limit

// Compositor modes (the dgs_mode values).
constexpr int kModeDuplex = 0;
constexpr int kModeAlpha = 1;
constexpr int kModeLcwsr = 2;

// Device-side error flags: bit n of the error word set for dgs_status n.
// A timed-out wait also sets a bit naming the kernel that gave up.
constexpr int kErrInvalid = 1;  // malformed cell_offsets
constexpr int kErrCapacity = 3;
constexpr int kErrTimeout = 6;
constexpr int kErrWaitScan = 8;  // the exclusive scan's look-back
constexpr int kErrWaitSort = 9;  // a radix sort pass's look-back

// Per-frame camera constants, passed by value to kernels.
struct CamK {
    float R[9], t[3];     // world -> camera
    float fx, fy, cx, cy;
    float znear;
    float o[3];           // camera centre, -R^T t
    double Rd[9], td[3];  // the same rotation/translation in binary64
    int W, H, TX, TY;
};

struct OptK {
    float eps, alpha_max, log2_alpha_min, delta, kappa;
    float bg[3];
    int v_one, no_et, stats;
    float tau;  // > 0: LC-WSR cell weights v max(0, 1 - depth / tau) instead of the cell transmittance
};

// Camera and options of one frame.  Kernels read them from device memory
// (written once per frame, or copied in before a captured graph is replayed)
// so that a captured frame can be replayed with a different camera.
struct FrameK {
    CamK k;
    OptK o;
    float* color;  // outputs of the frame ([3][H][W], [H][W] x 3; D, T, last nullable)
    float* D;
    float* T;
    int32_t* last;
    // a saved Duplex frame's own per-pixel state for its backward (null when
    // the frame is not saved): colour [3][H][W], D, and the replay start --
    // 1 + list position of the last contributing cell whose transmittance in
    // front is at least kMinReplayT -- with that transmittance
    float* sv_color;
    float* sv_D;
    float* sv_T;
    int32_t* sv_last;
};

// The backward recovers the transmittance in front of each replayed cell
// from the one behind it, T_n = T_{n+1} / P_n.  It starts at a cell whose own
// front transmittance the forward stored, and every cell in front of that
// one had a front transmittance >= kMinReplayT, so each P_n >= kMinReplayT
// and the division neither overflows nor meets 0/0.  Cells behind the
// replay start (only reachable with termination off or eps below this
// bound) carry weights below 2^-64 and are held at zero gradient.
constexpr float kMinReplayT = 0x1p-64f;

// Projected Gaussian as the compositor reads it (48 bytes).
//   dx = (px - x0) + ox, dy = (py - y0) + oy      (pixel offset from the mean)
//   log2(sigma G') = lo + ca dx^2 + cb dx dy + cc dy^2
//   inside the box  <=>  (unsigned)(px - x0) <= wx  and  (unsigned)(py - y0) <= wy
struct __align__(16) GRec {
    float ox, oy;
    float ca, cb, cc, lo;
    float r, g, b;
    int32_t x0, y0;
    uint32_t wxy;  // wx | wy << 16 (each <= 32767); culled: x0 = y0 = 0x7fff0000, wxy = 0
};
static_assert(sizeof(GRec) == 48, "GRec layout");

// log2 of a cell weight v in [0, 1] as the Duplex compositor folds it into
// its members' log2 sigma (forward and backward alike), floored at -126 so
// that v = 0 stays finite: a weight that small contributes nothing.
__device__ inline float fold_log2_weight(float v) { return fmaxf(__builtin_amdgcn_logf(v), -126.0f); }

// Look-back status words carry a 30-bit epoch (never 0) derived from a
// device-side frame counter (bumped by the per-frame clear kernel) and the
// pass index j < 16, so status buffers are zeroed once at allocation and
// never again, also when a captured frame is replayed.
__device__ inline uint32_t epoch_tag(uint32_t frame, uint32_t j) {
    return 1u + (uint32_t)(((uint64_t)frame * 16u + j) % ((1u << 30) - 1u));
}

// Packed integer rectangle: x0 | x1 << 16 | y0 << 32 | y1 << 48 (each < 2^15).
__host__ __device__ inline uint64_t pack_rect(int x0, int x1, int y0, int y1) {
    return (uint64_t)(uint16_t)x0 | ((uint64_t)(uint16_t)x1 << 16) | ((uint64_t)(uint16_t)y0 << 32) |
           ((uint64_t)(uint16_t)y1 << 48);
}
__host__ __device__ inline int rect_x0(uint64_t r) { return (int)(r & 0xffff); }
__host__ __device__ inline int rect_x1(uint64_t r) { return (int)((r >> 16) & 0xffff); }
__host__ __device__ inline int rect_y0(uint64_t r) { return (int)((r >> 32) & 0xffff); }
__host__ __device__ inline int rect_y1(uint64_t r) { return (int)((r >> 48) & 0xffff); }
constexpr uint64_t kEmptyRect = ~0ull;

// Workgroups are dispatched round-robin over the XCDs (block b runs on XCD
// b % 8).  Give each XCD one contiguous range of logical blocks so that
// neighbouring tiles, which share cells, share that XCD's L2.
__device__ inline int xcd_remap(int b, int nblocks) {
    int x = b % kXcds, local = b / kXcds;
    int per = nblocks / kXcds, rem = nblocks % kXcds;
    int base = x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per;
    return base + local;
}

}  // namespace dgs
