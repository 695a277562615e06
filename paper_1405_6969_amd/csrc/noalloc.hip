// noalloc.hip -- erpp_bin_static: the exact cell binning of erpp_bin for callers
// that cannot allocate device memory (code under stream capture, serving loops,
// harnesses that forbid hipMalloc).  Its scratch -- the cell histogram, the
// particle ranks and the scan partials -- lives in the file-scope array
// `scratch` below, one copy per GPU, held until the process ends.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "erpp_internal.hpp"

namespace {

// Largest box the static scratch holds.
constexpr int64_t kStaticMaxCells = int64_t(1) << 21;       // e.g. 128^3
constexpr int64_t kStaticMaxParticles = int64_t(1) << 21;
// Layout in 32-bit words: scan partials, histogram, ranks (each region starts on
// a 256-byte boundary).
constexpr int64_t kPartOff = 0;
constexpr int64_t kPartWords = kStaticMaxCells / erpp::kScanChunk + 64;
constexpr int64_t kCountOff = kPartOff + kPartWords;
constexpr int64_t kRankOff = kCountOff + kStaticMaxCells;
constexpr int64_t kScratchWords = kRankOff + kStaticMaxParticles;
static_assert(kPartWords % 64 == 0 && kCountOff % 64 == 0 && kRankOff % 64 == 0,
              "256-byte aligned regions");

// Device scratch of erpp_bin_static.  In host code `scratch` names a host-side
// stand-in, not device memory: kernels and copies receive the address that
// hipGetSymbolAddress returns for the current device (scratch_on_device).
static __device__ __align__(256) int32_t scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
int32_t *g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device
// (with that device current).
erpp_status scratch_on_device(int32_t **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return erpp::hip_fail(e, "erpp_bin_static: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return erpp::fail(ERPP_EUNSUPPORTED, "erpp_bin_static: device %d beyond %d", dev,
                          kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return erpp::hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                  "erpp_bin_static: hipGetSymbolAddress(scratch)");
        g_ptr[dev] = (int32_t *)p;
    }
    *out = g_ptr[dev];
    return ERPP_OK;
}

}  // namespace

extern "C" erpp_status erpp_bin_static(const int32_t n[3], const double L[3], int64_t np,
                                       const double *pos, int32_t *key, int32_t *perm,
                                       int32_t *bin_start, void *stream) {
    if (!n || !L) return erpp::fail(ERPP_EINVAL, "erpp_bin_static: n or L is NULL");
    erpp::BinGeom G;
    int64_t ncell = 1;
    for (int d = 0; d < 3; ++d) {
        if (n[d] < 1) return erpp::fail(ERPP_EINVAL, "erpp_bin_static: n[%d] = %d < 1", d, n[d]);
        if (!(L[d] > 0.0) || !std::isfinite(L[d]))
            return erpp::fail(ERPP_EINVAL, "erpp_bin_static: L[%d] must be finite and > 0", d);
        G.n[d] = n[d];
        G.L[d] = L[d];
        G.dx[d] = L[d] / (double)n[d];
        ncell *= n[d];
        if (ncell > kStaticMaxCells)
            return erpp::fail(ERPP_EINVAL,
                              "erpp_bin_static: %lld cells or more exceed the static scratch "
                              "(at most %lld cells)", (long long)ncell,
                              (long long)kStaticMaxCells);
    }
    if (np < 0 || np > kStaticMaxParticles)
        return erpp::fail(ERPP_EINVAL,
                          "erpp_bin_static: np = %lld outside [0, %lld] (static scratch)",
                          (long long)np, (long long)kStaticMaxParticles);
    if (!bin_start) return erpp::fail(ERPP_EINVAL, "erpp_bin_static: bin_start is NULL");
    if (np > 0 && (!pos || !key || !perm))
        return erpp::fail(ERPP_EINVAL, "erpp_bin_static: pos, key or perm is NULL");
    G.np = np;
    int32_t *base = nullptr;
    erpp_status s = scratch_on_device(&base);
    if (s != ERPP_OK) return s;
    // the histogram starts from zero on every call (a call that ended early may
    // have left it dirty)
    hipError_t e = erpp::bin_positions(G, pos, key, perm, bin_start, base + kCountOff,
                                       base + kRankOff, base + kPartOff, true,
                                       (hipStream_t)stream);
    if (e != hipSuccess) return erpp::hip_fail(e, "erpp_bin_static launch");
    return ERPP_OK;
}
