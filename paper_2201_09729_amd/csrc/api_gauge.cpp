// C ABI: version, errors, gauge handles, the full operator and kernel timing.
#include <cmath>
#include <cstring>

#include "../../include/dlma.h"
#include "runtime.h"

namespace dlma {
const char* last_error();
}

using namespace dlma;

static inline hipStream_t S(void* s) { return (hipStream_t)s; }

extern "C" const char* dlma_version(void) { return "dlma 0.1 gfx950"; }
extern "C" const char* dlma_last_error(void) { return dlma::last_error(); }

static int check_dims(const int* dims) {
    if (!dims) return fail(DLMA_EINVAL, "dims is NULL");
    long V = 1;
    for (int i = 0; i < 4; ++i) {
        if (dims[i] < 2 || (dims[i] & 1) || dims[i] > 4096)
            return fail(DLMA_EINVAL, "every lattice extent must be even, >= 2 and <= 4096 (extent " + std::to_string(i) + " = " +
                                         std::to_string(dims[i]) + ")");
        V *= dims[i];
        if (V >= (1L << 24)) return fail(DLMA_EINVAL, "lattice volume must be below 2^24 sites");
    }
    return DLMA_OK;
}

static int invert_clover(Gauge* g, hipStream_t s) {
    Buf err;
    DLMA_TRY(err.allocate(sizeof(int)));
    DLMA_HIP(hipMemsetAsync(err.p, 0, sizeof(int), s));
    DLMA_HIP(launch_clover_invert(g->Cl64[1].as<double2>(), g->Ci64.as<double2>(), g->Vh, err.as<int>(), s));
    int h = 0;
    DLMA_HIP(hipMemcpyAsync(&h, err.p, sizeof(int), hipMemcpyDeviceToHost, s));
    DLMA_HIP(hipStreamSynchronize(s));
    if (h) return fail(DLMA_EINVAL, "clover block not positive definite (kappa/csw out of range for this field)");
    for (int p = 1; p < 4; ++p) g->lo_ready[p] = false;
    return DLMA_OK;
}

extern "C" int dlma_load_gauge(const int dims[4], const void* U_dev, double kappa, double csw, void* stream,
                               dlma_gauge_t* out) {
    DLMA_TRY(check_dims(dims));
    if (!U_dev || !out) return fail(DLMA_EINVAL, "NULL gauge or output pointer");
    if (!(kappa > 0.0) || !std::isfinite(kappa)) return fail(DLMA_EINVAL, "kappa must be positive and finite");
    if (!(csw >= 0.0) || !std::isfinite(csw)) return fail(DLMA_EINVAL, "csw must be >= 0 and finite");
    hipStream_t s = S(stream);
    Gauge* g = new Gauge();
    for (int i = 0; i < 4; ++i) g->dims[i] = dims[i];
    g->geo = make_geo(dims);
    g->V = (long)dims[0] * dims[1] * dims[2] * dims[3];
    g->Vh = (int)(g->V / 2);
    g->kappa = kappa;
    g->csw = csw;
    auto bad = [&](int rc) { delete g; return rc; };
    const double2* Uc = (const double2*)U_dev;
    // unitarity and finiteness of every link
    {
        long nlink = g->V * 4;
        int nblk = ceil_div(nlink, 256);
        Buf bm;
        if (int rc = bm.allocate(sizeof(double) * nblk)) return bad(rc);
        if (launch_unitarity(Uc, nlink, bm.as<double>(), nblk, s) != hipSuccess) return bad(fail(DLMA_EHIP, "unitarity kernel launch failed"));
        std::vector<double> h(nblk);
        if (hipMemcpyAsync(h.data(), bm.p, sizeof(double) * nblk, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return bad(fail(DLMA_EHIP, "reading the unitarity check failed"));
        double m = 0;
        for (double v : h) m = std::max(m, v);
        if (!(m <= 1e-10)) return bad(fail(DLMA_EINVAL, "links are not unitary to 1e-10 (max |U U^dag - 1| = " + std::to_string(m) + ")"));
    }
    if (int rc = g->U64.allocate(sizeof(double2) * 2L * 4 * 9 * g->Vh)) return bad(rc);
    if (int rc = g->Cl64[0].allocate(sizeof(double2) * 2L * 18 * g->Vh)) return bad(rc);
    if (int rc = g->Cl64[1].allocate(sizeof(double2) * 2L * 18 * g->Vh)) return bad(rc);
    if (int rc = g->Ci64.allocate(sizeof(double2) * 2L * 18 * g->Vh)) return bad(rc);
    if (launch_pack_links(Uc, g->U64.as<double2>(), g->geo, s) != hipSuccess) return bad(fail(DLMA_EHIP, "link packing failed"));
    double m0 = 1.0 / (2.0 * kappa) - 4.0;
    if (launch_clover_build(Uc, g->geo, m0, csw, g->Cl64[0].as<double2>(), g->Cl64[1].as<double2>(), s) != hipSuccess)
        return bad(fail(DLMA_EHIP, "clover construction failed"));
    if (int rc = invert_clover(g, s)) return bad(rc);
    *out = (dlma_gauge_t)g;
    return DLMA_OK;
}

extern "C" int dlma_set_mass(dlma_gauge_t h, double kappa, void* stream) {
    Gauge* g = (Gauge*)h;
    if (!g) return fail(DLMA_EINVAL, "NULL handle");
    if (!(kappa > 0.0) || !std::isfinite(kappa)) return fail(DLMA_EINVAL, "kappa must be positive and finite");
    hipStream_t s = S(stream);
    double delta = (1.0 / (2.0 * kappa)) - (1.0 / (2.0 * g->kappa));
    DLMA_HIP(launch_add_diag(g->Cl64[0].as<double2>(), g->Vh, delta, s));
    DLMA_HIP(launch_add_diag(g->Cl64[1].as<double2>(), g->Vh, delta, s));
    g->kappa = kappa;
    return invert_clover(g, s);
}

extern "C" int dlma_free_gauge(dlma_gauge_t h) {
    Gauge* g = (Gauge*)h;
    if (!g) return fail(DLMA_EINVAL, "NULL handle");
    (void)hipDeviceSynchronize();
    delete g;
    return DLMA_OK;
}

extern "C" int dlma_gauge_info(dlma_gauge_t h, int dims_out[4], double* kappa_out, double* csw_out) {
    Gauge* g = (Gauge*)h;
    if (!g) return fail(DLMA_EINVAL, "NULL handle");
    if (dims_out)
        for (int i = 0; i < 4; ++i) dims_out[i] = g->dims[i];
    if (kappa_out) *kappa_out = g->kappa;
    if (csw_out) *csw_out = g->csw;
    return DLMA_OK;
}

// y = D x (or g5 D g5 x) on full FP64 even-odd fields, both parities in one launch
int apply_full64(Gauge* g, void* in_eo, void* out_eo, int nrhs, int dagger, hipStream_t s) {
    std::vector<HopJob<P64>> jobs;
    for (int par = 0; par < 2; ++par) {
        HopJob<P64> j = hop_job<P64>(g, par, nrhs, 1);
        j.U = g->U64.as<double2>();
        j.C = g->Cl64[par].as<double2>();
        j.x = full_view(in_eo, g->Vh, par);
        j.in = full_view(in_eo, g->Vh, 1 - par);
        j.out = full_view(out_eo, g->Vh, par);
        j.ca = 1.0;
        j.ch = -0.5;
        jobs.push_back(j);
    }
    int nblk = assign_blocks(jobs);
    Buf dj;
    DLMA_TRY(dj.allocate(sizeof(HopJob<P64>) * jobs.size()));
    DLMA_HIP(hipMemcpyAsync(dj.p, jobs.data(), sizeof(HopJob<P64>) * jobs.size(), hipMemcpyHostToDevice, s));
    HopCfg c{K2, dagger ? (F_G5IN | F_G5OUT) : 0, 1};
    DLMA_HIP(launch_hop<P64>(c, dj.as<HopJob<P64>>(), (int)jobs.size(), nblk, s));
    DLMA_HIP(hipStreamSynchronize(s));
    return DLMA_OK;
}

extern "C" int dlma_apply_dw(dlma_gauge_t h, const void* in, void* out, int nrhs, int dagger, void* stream) {
    Gauge* g = (Gauge*)h;
    if (!g) return fail(DLMA_EINVAL, "NULL handle");
    if (nrhs < 0) return fail(DLMA_EINVAL, "nrhs < 0");
    if (nrhs == 0) return DLMA_OK;
    if (!in || !out) return fail(DLMA_EINVAL, "NULL field pointer");
    if (in == out) return fail(DLMA_EINVAL, "in and out must not overlap");
    hipStream_t s = S(stream);
    size_t bytes = sizeof(double2) * (size_t)nrhs * 24 * g->Vh;
    Buf a, b;
    DLMA_TRY(a.allocate(bytes));
    DLMA_TRY(b.allocate(bytes));
    DLMA_HIP(launch_canon_to_eo((const double2*)in, a.as<double2>(), g->geo, nrhs, s));
    DLMA_TRY(apply_full64(g, a.p, b.p, nrhs, dagger, s));
    DLMA_HIP(launch_eo_to_canon(b.as<double2>(), (double2*)out, g->geo, nrhs, s));
    DLMA_HIP(hipStreamSynchronize(s));
    return DLMA_OK;
}

// ---------------------------------------------------------------- timing

extern "C" int dlma_profile_enable(int on) {
    Profiler::get().on = on != 0;
    return DLMA_OK;
}

extern "C" int dlma_profile_reset(void) {
    Profiler& p = Profiler::get();
    for (int k = 0; k < KC_N; ++k) {
        p.launches[k] = 0;
        p.ms[k] = 0;
        p.bytes[k] = 0;
    }
    return DLMA_OK;
}

extern "C" int dlma_profile_read(int kc, long long* launches, double* total_ms, double* total_bytes) {
    if (kc < 0 || kc >= KC_N) return fail(DLMA_EINVAL, "kernel class out of range");
    Profiler& p = Profiler::get();
    if (launches) *launches = p.launches[kc];
    if (total_ms) *total_ms = p.ms[kc];
    if (total_bytes) *total_bytes = p.bytes[kc];
    return DLMA_OK;
}
