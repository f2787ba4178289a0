// qlra_noalloc(): the solve of qlra() for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid allocation).  Its workspace is a
// file-scope device array instead of a caller buffer; nothing is allocated, no stream, event or
// graph is created (the per-pass estimates run on the caller's stream).
#include <mutex>

#include "common.h"
#include "qlra_noalloc.h"

namespace qlra_impl {
namespace {

// 128 MiB: every FP32 solve of the serving mix (m, n <= 2048, k + p <= 80, v <= 6, either
// scheme) fits; qlra_workspace_size() tells whether a given solve does.
constexpr size_t kScratchBytes = (size_t)128 << 20;

// One copy per device, held until the process ends.  Host code never uses this name as an
// address: the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's scratch array (looked up on the first call on a device).
int scratch_on_current_device(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return QLRA_E_HIP;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return QLRA_E_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return QLRA_OK;
}

}  // namespace
}  // namespace qlra_impl

extern "C" {

size_t qlra_noalloc_max_bytes(void) { return qlra_impl::kScratchBytes; }

int qlra_noalloc(const float* A, int64_t m, int64_t n, int64_t lda, int64_t a_plane_stride, int k, int p,
                 int pass_budget, int scheme, uint64_t seed, const qlra_opts_t* opts, float* U, int64_t ldu,
                 int64_t u_plane_stride, double* S, float* V, int64_t ldv, int64_t v_plane_stride, double* pass_err) {
    if (!opts) return QLRA_E_ARG;
    size_t need = 0;
    int rc = qlra_workspace_size(m, n, k, p, pass_budget, scheme, opts, &need);
    if (rc != QLRA_OK) return rc;
    if (need > qlra_impl::kScratchBytes) return QLRA_E_TOO_LARGE;
    void* ws = nullptr;
    if ((rc = qlra_impl::scratch_on_current_device(&ws)) != QLRA_OK) return rc;
    qlra_opts_t o = *opts;
    o.workspace = ws;
    o.workspace_bytes = qlra_impl::kScratchBytes;
    o.graph = 0;
    return qlra_impl::solve_entry(A, m, n, lda, a_plane_stride, k, p, pass_budget, scheme, seed, &o, U, ldu,
                                  u_plane_stride, S, V, ldv, v_plane_stride, pass_err, true);
}

int qlra_noalloc_status(void* stream, int* status) {
    void* ws = nullptr;
    const int rc = qlra_impl::scratch_on_current_device(&ws);
    if (rc != QLRA_OK) return rc;
    return qlra_status(ws, stream, status);
}

}  // extern "C"
