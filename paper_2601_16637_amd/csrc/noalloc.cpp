// sigma = (H - shift) c with no device allocation: the workspace of the
// matrix-free product lives in a static device array of fixed size instead of
// a buffer the Hamiltonian handle allocates per stream.  For callers that may
// not allocate (code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc).
//
// Each GPU the library runs on holds its own copy of the array from the first
// call on that device until the process ends.  Every call on a device shares
// that copy, so calls that overlap on one device (on different streams, or
// from several threads) race on it; calls ordered on one stream do not.  The
// array keeps the previous call's contents; nothing needs clearing, since the
// product writes every workspace element it later reads (the transposed input
// and the beta-side partial result) before reading it.
#include <mutex>

#include "internal.h"

using namespace sbd;

namespace {

constexpr int kMaxDevices = 64;

// In host code `scratch` is only a stand-in for the device symbol: its device
// address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[SBD_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (looked up on the
// first call on that device, with the device current).
int scratch_address(void** out) {
    int dev = -1;
    SBD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SBD_ERR_ARG, "sbd_sigma_noalloc: device ordinal out of range");
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(SBD_ERR_HIP, "hipGetSymbolAddress(scratch) returned a null address");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return SBD_OK;
}

}  // namespace

extern "C" int sbd_sigma_noalloc(const sbd_basis* b, const sbd_exc* x, const sbd_ham* H, int nvec, int prec,
                                 double shift, const void* c, void* sigma, int layout, void* stream) {
    int rc = sigma_validate(b, x, H, nvec, prec, shift, c, sigma, layout);
    if (rc) return rc;
    const int64_t N = H->na * H->nb;
    void* ws = nullptr;
    if (!H->csr_has[prec == SBD_FP64 ? 0 : 1] && N > 0) {  // the CSR product needs no workspace
        const size_t need = sigma_workspace_bytes(N, nvec, layout, prec == SBD_FP64 ? 8 : 4);
        if (need > (size_t)SBD_NOALLOC_SCRATCH_BYTES)
            return fail(SBD_ERR_NOMEM, "sbd_sigma_noalloc: this product needs " + std::to_string(need) +
                                           " bytes of workspace; the static scratch holds " +
                                           std::to_string((size_t)SBD_NOALLOC_SCRATCH_BYTES));
        rc = scratch_address(&ws);
        if (rc) return rc;
    }
    return sigma_internal(x, H, nvec, prec, shift, c, sigma, layout, ws, (hipStream_t)stream);
}
