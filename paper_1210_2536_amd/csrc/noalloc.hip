// Allocation-free feature extraction: spmv_features_compute with every
// device buffer (validation flags, row and entry statistics, the diagonal
// histogram of the census and the row-degree histogram of the power-law
// fit) carved out of one fixed device array instead of allocated.
//
// The array is a file-scope __device__ variable: each GPU the library runs
// on holds its own copy, at its own address, until the process ends.  Host
// code never uses the array's name as a device address: the address is
// looked up once per device with hipGetSymbolAddress and that pointer is
// what the kernels and memsets receive.  Every call on a device shares the
// array; the feature pass clears what it accumulates into (its scratch
// block by a kernel, its histograms by memsets) before use, so a call never
// sees the previous call's counts, but two calls that overlap on one device
// race.
#include <mutex>

#include "internal.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// The calling thread's current device's copy of `scratch`, looked up once.
spmv_status scratch_ptr(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return smat::hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) {
        smat::set_error("device %d beyond the %d devices the fixed scratch serves", dev,
                        kMaxDevices);
        return SPMV_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return smat::hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                  "hipGetSymbolAddress(scratch)");
        }
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return SPMV_OK;
}

}  // namespace

extern "C" spmv_status spmv_features_compute_noalloc(const spmv_csr *A, spmv_features *out,
                                                     void *stream) {
    if (A && A->m >= 0 && A->n >= 0 && A->m < INT32_MAX && A->n < INT32_MAX &&
        smat::features_region_bytes(A->m, A->n) > kScratchBytes) {
        smat::set_error("spmv_features_compute_noalloc: an %lld x %lld matrix needs %zu bytes "
                        "of scratch, above the fixed %zu (256 + 4 (m + n - 1) + 4 (n + 2) "
                        "bytes, each part rounded up to 256)",
                        (long long)A->m, (long long)A->n, smat::features_region_bytes(A->m, A->n),
                        kScratchBytes);
        return SPMV_EUNSUPPORTED;
    }
    void *p = nullptr;
    spmv_status st = scratch_ptr(&p);
    if (st != SPMV_OK) return st;
    return smat::features_in_region(A, out, (hipStream_t)stream, p, kScratchBytes);
}
