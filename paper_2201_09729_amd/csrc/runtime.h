// Host runtime of the dlma library: error state, device memory pool, gauge
// handle, kernel-timing registry.
#pragma once
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dlma.h"
#include "kernels.h"

namespace dlma {

// ---------------------------------------------------------------- errors

void set_error(const std::string& m);
int fail(int code, const std::string& m);

#define DLMA_HIP(expr)                                                                          \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return ::dlma::fail(DLMA_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define DLMA_TRY(expr)          \
    do {                        \
        int rc_ = (expr);       \
        if (rc_ != 0) return rc_; \
    } while (0)

// ---------------------------------------------------------------- device memory

// Size-keyed cache of device allocations.  Blocks are returned only after the
// stream that used them has been synchronised, so reuse never races.
class Pool {
  public:
    static Pool& get();
    void* alloc(size_t bytes);
    void release(void* p, size_t bytes);
    void trim();

  private:
    std::mutex m_;
    std::multimap<size_t, void*> free_;
};

// RAII device buffer from the pool
struct Buf {
    void* p = nullptr;
    size_t n = 0;
    Buf() = default;
    Buf(const Buf&) = delete;
    Buf& operator=(const Buf&) = delete;
    Buf(Buf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    Buf& operator=(Buf&& o) noexcept {
        if (this != &o) {
            reset();
            p = o.p; n = o.n;
            o.p = nullptr; o.n = 0;
        }
        return *this;
    }
    ~Buf() { reset(); }
    int allocate(size_t bytes);  // DLMA_OK or DLMA_ENOMEM
    void reset() {
        if (p) Pool::get().release(p, n);
        p = nullptr;
        n = 0;
    }
    template <class T> T* as() const { return (T*)p; }
};

// ---------------------------------------------------------------- gauge handle

struct Gauge {
    int dims[4];
    Geo geo;
    long V;
    int Vh;
    double kappa, csw;
    Buf U64;        // [2][4][9][Vh] double2
    Buf Cl64[2];    // A per parity, [2][18][Vh] double2
    Buf Ci64;       // A_oo^-1, [2][18][Vh] double2
    Buf Ulo[4];     // links in P32 / P16 / PB16 (index = precision)
    Buf Cee[4];     // A_ee in that precision
    Buf Cio[4];     // A_oo^-1 in that precision
    bool lo_ready[4] = {false, false, false, false};
};

// Autotuner results, shared by all handles: (T, Z, Y, X, precision, nrhs) -> right-hand sides per thread
int tuned_lookup(const int dims[4], int prec, int nrhs);
void tuned_store(const int dims[4], int prec, int nrhs, int nb);

int gauge_prepare(Gauge* g, int prec, hipStream_t s);  // low-precision copies on demand
const void* gauge_links(const Gauge* g, int prec);
const void* gauge_clover_ee(const Gauge* g, int prec);
const void* gauge_clover_oo_inv(const Gauge* g, int prec);

// ---------------------------------------------------------------- stencil jobs

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// site blocks of a stencil launch: whole blocks per timeslice (see the block decode)
inline int hop_nsb(const Geo& g) { return g.T * ceil_div(g.Z * g.Y * g.Xh, HOP_BS); }

// window: FP16 stencils may stage the +-x, +-y neighbours through LDS (when they fit)
template <int P> HopJob<P> hop_job(const Gauge* g, int par, int nrhs, int nb, bool window = true) {
    HopJob<P> j = {};
    j.g = g->geo;
    j.par = par;
    j.nrhs = nrhs;
    j.G = ceil_div(nrhs, nb);
    j.vt = g->geo.Z * g->geo.Y * g->geo.Xh;
    j.nbt = ceil_div(j.vt, HOP_BS);
    j.nsb = hop_nsb(g->geo);
    j.nxb = ceil_div(g->geo.T, 8) * j.nbt;
    j.pstride = j.nsb;
    // FP16 stencils: the block's sites and one y row on either side, if LDS has room
    const int wn = HOP_BS + 2 * g->geo.Xh;
    j.wn = (window && P == P16 && (int)hop_window_bytes(nb, wn) <= hop_window_max_bytes(nb)) ? wn : 0;
    return j;
}

// assign consecutive workgroup ranges; returns the total number of workgroups
// workgroups of a stencil launch of one job restricted to twn timeslices (HopCfg)
inline int hop_window_blocks(const Geo& g, int nrhs, int nb, int twn) {
    return 8 * ceil_div(twn, 8) * ceil_div(g.Z * g.Y * g.Xh, HOP_BS) * ceil_div(nrhs, nb);
}

template <int P> int assign_blocks(std::vector<HopJob<P>>& jobs) {
    int b = 0;
    for (auto& j : jobs) {
        j.blk0 = b;
        b += 8 * j.nxb * j.G;
    }
    return b;
}

template <int P> int assign_vec_blocks(std::vector<VecJob<P>>& jobs) {
    int b = 0;
    for (auto& j : jobs) {
        j.blk0 = b;
        b += j.nsb * j.nrhs;
    }
    return b;
}

// half-field view helpers
template <int P> SF<P> half_view(void* base, float* nrm, int Vh, int r0 = 0) {
    SF<P> f;
    f.rs = 12L * Vh;
    f.ns = Vh;
    f.v = (typename PT<P>::S*)base + (size_t)r0 * f.rs;
    f.nrm = nrm ? nrm + (size_t)r0 * Vh : nullptr;
    return f;
}
// parity half of a full FP64 field [rhs][2][12][Vh]
inline SF<P64> full_view(void* base, int Vh, int par) {
    SF<P64> f;
    f.rs = 24L * Vh;
    f.ns = 0;
    f.v = (double2*)base + (size_t)par * 12 * Vh;
    f.nrm = nullptr;
    return f;
}

// algorithmic (compulsory) bytes of one stencil launch for one job
double hop_bytes(int prec, int kind, int flags, int Vh, int nrhs_active);

// ---------------------------------------------------------------- timing registry

enum KClass {
    KC_K1 = 0, KC_K1DAG = 1, KC_K2DAGN = 2, KC_K2CG = 3, KC_K2 = 4,  // stencils
    KC_LAP_MATVEC = 5,  // Lanczos: applications of -lap (or of its Chebyshev polynomial); block: the filter
    KC_LAP_ORTHO = 6,   // Lanczos: three-term step, two Gram-Schmidt passes, normalisation; block: Cholesky QR
    KC_LAP_RITZ = 7,    // Lanczos: Ritz vectors and Rayleigh-quotient residual checks; block: Rayleigh-Ritz
    KC_K2V = 8,         // BiCGStab: v = Dhat p (K2 with (rh, v))
    KC_K2T = 9,         // BiCGStab: t = Dhat s (K2 with (t, s), |t|^2)
    KC_N = 10
};

struct Profiler {
    static Profiler& get();
    bool on = false;
    long long launches[KC_N] = {};
    double ms[KC_N] = {};
    double bytes[KC_N] = {};
    // pending event pairs for the current call
    struct Pending { hipEvent_t a, b; int kc; double bytes; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> spare;
    std::mutex m;
    hipEvent_t ev();
    void begin(int kc, double bytes, hipStream_t s, hipEvent_t& a);
    void end(hipEvent_t a, int kc, double bytes, hipStream_t s);
    void collect();  // after the stream is synchronised
};

}  // namespace dlma
