// mdn_denoise_noalloc: the whole cascade of mdn_denoise with its workspace in a static device
// array instead of caller memory, for callers that cannot allocate (code under HIP graph capture,
// tight serving loops).
//
// The array is a file-scope __device__ symbol: the code object reserves it on every device the
// library is loaded on, and it lives until the process ends. Host code never passes its name to a
// kernel (in host code the name is only a host-side stand-in); the device address comes from
// hipGetSymbolAddress, looked up once per device on the first call made with that device current.
#include <mutex>

#include "mdn_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)MDN_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[MDN_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (nullptr and an error set on failure).
void* scratch_on_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        mdn::fail(MDN_EDEVICE, "noalloc: no current device (or device index >= %d)", kMaxDevices);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            mdn::fail(MDN_EDEVICE, "noalloc: hipGetSymbolAddress of the scratch array failed on device %d: %s", dev,
                      hipGetErrorString(e));
            return nullptr;
        }
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

}  // namespace

extern "C" mdn_status mdn_denoise_noalloc(const mdn_image* in, const mdn_bank* bank, int32_t storage,
                                          const mdn_image* out, void* stream) {
    mdn::clear_error();
    if (!in || !bank || !out) return mdn::fail(MDN_EINVAL, "null argument");
    if (!bank->level || bank->levels < 1 || bank->levels > 16) return mdn::fail(MDN_EINVAL, "bank: need 1..16 levels");
    size_t need = 0;
    mdn_status st = mdn_denoise_workspace_size(in->width, in->height, in->channels, bank->levels, storage, &need);
    if (st) return st;
    if (need > kScratchBytes)
        return mdn::fail(MDN_ENOMEM, "noalloc: the cascade needs %zu bytes of workspace, above the static scratch "
                                     "of %zu bytes (use mdn_denoise with a caller workspace)",
                         need, kScratchBytes);
    void* ws = scratch_on_current_device();
    if (!ws) return MDN_EDEVICE;
    // every byte the cascade reads from the workspace is written earlier in the same call (pyramid
    // levels, coarser outputs and selector maps), so nothing needs clearing between calls
    return mdn_denoise(in, bank, storage, ws, kScratchBytes, out, stream);
}
