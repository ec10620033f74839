// Allocation-free forward: wn_voxelize_strips with its workspace in a fixed,
// file-scope device array instead of a caller-supplied buffer, for callers that
// cannot allocate device memory (code under stream capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// The array holds what the workspace of wn_voxelize_strips holds: the header with the
// device error record, the vertex records of the stream and the per-split partial sums.
// Every GPU the library runs on keeps its own copy of the array until the process ends.
// In host code the array's name is not a device address, so each device's address is
// taken once with hipGetSymbolAddress (with that device current) and kept; only that
// address is ever passed to kernels or copies.
#include <mutex>

#include "wn_internal.hpp"

static __device__ __align__(256) char scratch[WN_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kScratchBytes = WN_NOALLOC_SCRATCH_BYTES;  // per device
constexpr int kMaxDevices = 64;

std::mutex g_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch` on each device, once taken

// Device address of the scratch array on the current device (taken on first use).
wn_status scratch_address(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return WN_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return WN_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[dev] == nullptr) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return WN_ERR_HIP;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return WN_OK;
}

}  // namespace

namespace wn {

// The scratch header of the current device, for wn_get_device_error(NULL, ...).
wn_status noalloc_header(void **out) { return scratch_address(out); }

}  // namespace wn

extern "C" {

wn_status wn_voxelize_strips_noalloc(const float *V, int64_t nV, const int32_t *F, int64_t nF,
                                     const int32_t *strips, int64_t n_records, const wn_grid *grid,
                                     const float *Q, int64_t nQ, float *W, int32_t occ_mode, float tau, float k,
                                     void *occ, void *stream) {
    if (strips == nullptr) return WN_ERR_INVALID_ARG;
    void *ws = nullptr;
    const wn_status st = scratch_address(&ws);
    if (st != WN_OK) return st;
    // the same checks and launch sequence as wn_voxelize_strips; a stream whose
    // workspace exceeds the array returns WN_ERR_WORKSPACE before anything is enqueued
    return wn::voxelize_impl(V, nV, F, nF, strips, n_records, grid, Q, nQ, W, occ_mode, tau, k, occ, ws,
                             kScratchBytes, stream, nullptr);
}

}  // extern "C"
