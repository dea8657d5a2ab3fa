// Allocation-free variant of the distillation projector (dlma_project_noalloc).
//
// dlma_project takes its coefficient buffer c[r][k][s] = <v_k(t) x e_s, in_r>_t from
// the library's device pool.  Callers that may not allocate device memory (code
// under stream capture, serving loops) use this entry point instead: its
// coefficients live in one fixed device array per GPU, declared below, and the
// right-hand sides are processed in chunks that fit it.  The kernels are the same
// as dlma_project's, so the two give bit-identical results.
#include <mutex>

#include "laplace.h"
#include "runtime.h"

namespace dlma {

// Coefficient scratch: 65536 complex doubles (1 MiB) per GPU, held until the
// process ends.  Host code never uses this name as an address: it is a host-side
// stand-in.  The device address comes from hipGetSymbolAddress, once per device.
constexpr long kProjScratchPairs = 65536;
static __device__ __align__(256) double2 scratch[kProjScratchPairs];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double2* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on first use there).
int scratch_on_current_device(double2** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(DLMA_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(DLMA_EUNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> l(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(DLMA_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = (double2*)p;
    }
    *out = g_scratch_dev[dev];
    return DLMA_OK;
}

}  // namespace
}  // namespace dlma

using namespace dlma;

extern "C" int dlma_project_noalloc(dlma_gauge_t h, int t, int nev, const void* V_t, const void* in, void* out, int nrhs,
                                    int mode, void* stream) {
    Gauge* g = (Gauge*)h;
    if (!g) return fail(DLMA_EINVAL, "NULL handle");
    if (t < 0 || t >= g->dims[0]) return fail(DLMA_EINVAL, "timeslice out of range");
    if (mode != 0 && mode != 1) return fail(DLMA_EINVAL, "mode must be 0 or 1");
    if (nrhs < 0 || nev < 0) return fail(DLMA_EINVAL, "negative count");
    const long per_rhs = 4L * std::max(1, nev);  // coefficients of one right-hand side
    if (per_rhs > kProjScratchPairs)
        return fail(DLMA_EINVAL, "nev = " + std::to_string(nev) + " exceeds the allocation-free projector's limit of " +
                                     std::to_string(kProjScratchPairs / 4) + " modes");
    if (nrhs == 0) return DLMA_OK;
    if (!in || !out || (nev > 0 && !V_t)) return fail(DLMA_EINVAL, "NULL pointer");
    double2* coef = nullptr;
    DLMA_TRY(scratch_on_current_device(&coef));
    hipStream_t s = (hipStream_t)stream;
    const long fs = 12L * g->V;                         // complex numbers per spinor field
    const int chunk = (int)(kProjScratchPairs / per_rhs);  // right-hand sides per pass through the scratch
    for (int r0 = 0; r0 < nrhs; r0 += chunk) {
        const int nr = std::min(chunk, nrhs - r0);
        DLMA_HIP(launch_project((const double2*)V_t, (const double2*)in + (size_t)r0 * fs, (double2*)out + (size_t)r0 * fs,
                                g->geo, t, nev, nr, mode, coef, s));
    }
    return DLMA_OK;
}
