// dgs_sort_pairs_noalloc: the library's onesweep sort with its scratch
// memory in one static device array, for callers that cannot allocate.
//
// Every GPU the library runs on holds its own copy of `scratch` from module
// load until the process ends.  Host code never passes the array's name to
// a kernel (on the host it only stands in for the symbol): the device
// address is looked up once per device with hipGetSymbolAddress, with that
// device current, and kept in a per-device table.
#include <mutex>
#include <string>

#include "ctx.h"

using namespace dgs;

namespace {

constexpr int64_t kNoAllocMaxKeys = DGS_SORT_NOALLOC_MAX_KEYS;

// Layout of the scratch array (byte offsets, each part 256-byte aligned):
//   words  [64] u32: [0] look-back epoch counter, [1..8] pass tickets, [9] key count
//   hist   [8][256] u32 digit counts
//   keys   [kNoAllocMaxKeys] u64 and vals [kNoAllocMaxKeys] u32: the sort's ping-pong partner
//   status look-back words of every partition, u64
constexpr size_t kOffWords = 0;
constexpr size_t kOffHist = 256;
constexpr size_t kOffKeys = kOffHist + 8 * 256 * 4;
constexpr size_t kOffVals = kOffKeys + 8 * (size_t)kNoAllocMaxKeys;
constexpr size_t kOffStatus = kOffVals + 4 * (size_t)kNoAllocMaxKeys;
// 256 look-back words per partition of at least 1,024 keys
constexpr size_t kStatusWords = (size_t)((kNoAllocMaxKeys + 1023) / 1024) * 256;
constexpr size_t kScratchBytes = kOffStatus + 8 * kStatusWords;  // ~14.3 MB

// Zero at module load: epoch 0 (never used by a sort) in every status word.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_ptr[kMaxDevices] = {};

}  // namespace

// Looks up this device's copy of the scratch array (the device must be
// current); called once per device at context creation.
hipError_t dgs_internal_noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[device] = static_cast<unsigned char*>(p);
    return hipSuccess;
}

extern "C" {

dgs_status dgs_sort_pairs_noalloc(dgs_ctx c, uint64_t* keys, uint32_t* values, int64_t n, int32_t key_bits) {
    if (!c) return DGS_ERR_INVALID_ARG;
    if (n < 0 || key_bits < 1 || key_bits > 64) {
        c->err = "bad n or key_bits";
        return DGS_ERR_INVALID_ARG;
    }
    if (n > kNoAllocMaxKeys) {
        c->err = "dgs_sort_pairs_noalloc sorts at most " + std::to_string(kNoAllocMaxKeys) + " pairs, got " +
                 std::to_string(n);
        return DGS_ERR_INVALID_ARG;
    }
    if (n == 0) return DGS_OK;
    if (!keys || !values) {
        c->err = "NULL buffer";
        return DGS_ERR_INVALID_ARG;
    }
    unsigned char* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        base = g_ptr[c->device];
    }
    if (!base) {
        c->err = "no scratch address for this device (context creation failed to look it up)";
        return DGS_ERR_DEVICE;
    }
    hipSetDevice(c->device);
    uint32_t* words = reinterpret_cast<uint32_t*>(base + kOffWords);
    uint32_t* hist = reinterpret_cast<uint32_t*>(base + kOffHist);
    uint64_t* k1 = reinterpret_cast<uint64_t*>(base + kOffKeys);
    uint32_t* v1 = reinterpret_cast<uint32_t*>(base + kOffVals);
    uint64_t* status = reinterpret_cast<uint64_t*>(base + kOffStatus);
    // the array keeps the previous call's contents: the digit counts and
    // the pass tickets start at zero again (a kernel, no memset node), the
    // epoch counter moves on so that old look-back words are never read as
    // this call's
    ClearList cl;
    cl.add(hist, 8 * 256);
    cl.add(words + 1, 8);
    cl.bump = words + 0;
    launch_clear(c->stream, cl);
    launch_fill_u32(c->stream, words + 9, (uint32_t)n, 1);
    const SortScratch ss{hist, status, words + 1};
    const bool in1 = launch_radix_sort(c->stream, keys, values, k1, v1, words + 9, (uint32_t)n, key_bits, ss,
                                       words + 0, c->dev_err);
    if (in1) {
        hipMemcpyAsync(keys, k1, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, c->stream);
        hipMemcpyAsync(values, v1, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, c->stream);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        c->err = std::string("kernel launch failed: ") + hipGetErrorString(e);
        return DGS_ERR_DEVICE;
    }
    return DGS_OK;
}

}  // extern "C"
