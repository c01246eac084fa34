// goat_sinkhorn_noalloc: goat_sinkhorn for callers that cannot allocate
// device memory (code under graph capture, tight serving loops). The
// solve's small state (potentials, per-strip column partials, control
// block, reduction partials, warm-start features) lives in `scratch`, a
// static device array of kScratchBytes that every GPU the library runs on
// holds until the process ends; the caller passes only G and the outputs.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is taken once per device with hipGetSymbolAddress (with
// that device current) and only that address is passed to kernels.
#include <cstdint>
#include <mutex>

#include "common.h"

namespace goat {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call per device); GOAT_EHIP with the runtime's message on failure.
int scratch_address(void** out) {
    int dev = 0;
    GOAT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("goat_sinkhorn_noalloc: device index too large");
        return GOAT_ENOTSUP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        GOAT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GOAT_OK;
}

size_t scratch_need(int n) { return small_bytes(make_layout(n, GOAT_PREC_FP32, 1)); }

}  // namespace
}  // namespace goat

using namespace goat;

extern "C" {

size_t goat_sinkhorn_noalloc_scratch_bytes(void) { return kScratchBytes; }

int goat_sinkhorn_noalloc_max_n(void) {
    // the state grows with n (column partials of every strip); the largest n
    // whose state fits, found by bisection over the host-side layout
    int lo = 1, hi = 1 << 20;
    while (lo < hi) {
        const int mid = lo + (hi - lo + 1) / 2;
        if (scratch_need(mid) <= kScratchBytes) lo = mid; else hi = mid - 1;
    }
    return lo;
}

int goat_sinkhorn_noalloc(int n, const float* G, int ldg, const float* eps_dev, float eps_rel, float* f, float* g,
                          int init, const float* mlp_params, int max_iter, float tol, float* Q, int ldq,
                          int* iters_dev, float* err_dev, float* eps_out, void* stream) {
    clear_error();
    int rc = sinkhorn_check(n, G, ldg, eps_dev, eps_rel, g, init, mlp_params, max_iter, tol, Q, ldq);
    if (rc) return rc;
    if (scratch_need(n) > kScratchBytes) {
        set_error("goat_sinkhorn_noalloc: n exceeds goat_sinkhorn_noalloc_max_n() (the static scratch holds "
                  "64 MiB of solver state)");
        return GOAT_EINVAL;
    }
    if (sinkhorn_needs_repack(G, ldg, max_iter)) {
        set_error("goat_sinkhorn_noalloc: G must be 16-byte aligned with ldg a multiple of 4, and of 64 when "
                  "max_iter >= 8 (there is no space to repack it)");
        return GOAT_EINVAL;
    }
    void* base = nullptr;
    rc = scratch_address(&base);
    if (rc) return rc;
    const Layout L = make_layout(n, GOAT_PREC_FP32, 1);
    const Ptrs p = make_ptrs(L, base);
    return sinkhorn_run(n, G, ldg, eps_dev, eps_rel, f, g, init, mlp_params, max_iter, tol, Q, ldq, iters_dev,
                        err_dev, eps_out, p, L.np, false, static_cast<hipStream_t>(stream));
}

}  // extern "C"
