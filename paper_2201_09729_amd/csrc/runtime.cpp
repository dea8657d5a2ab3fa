// Host runtime: error state, device memory pool, gauge handle preparation,
// kernel-timing registry and the algorithmic byte model of the stencil launches.
#include "runtime.h"

namespace dlma {

static thread_local std::string t_err;

void set_error(const std::string& m) { t_err = m; }
int fail(int code, const std::string& m) {
    t_err = m;
    return code;
}
const char* last_error() { return t_err.c_str(); }

// ---------------------------------------------------------------- pool

Pool& Pool::get() {
    static Pool* p = new Pool();  // never destroyed: blocks live until process end
    return *p;
}

static size_t round_bytes(size_t b) {
    const size_t g = (size_t)1 << 20;
    return b < g ? ((b + 255) / 256) * 256 : ((b + g - 1) / g) * g;
}

void* Pool::alloc(size_t bytes) {
    bytes = round_bytes(bytes);
    {
        std::lock_guard<std::mutex> l(m_);
        auto it = free_.find(bytes);
        if (it != free_.end()) {
            void* p = it->second;
            free_.erase(it);
            return p;
        }
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        trim();
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    return p;
}

void Pool::release(void* p, size_t bytes) {
    std::lock_guard<std::mutex> l(m_);
    free_.emplace(round_bytes(bytes), p);
}

void Pool::trim() {
    std::multimap<size_t, void*> f;
    {
        std::lock_guard<std::mutex> l(m_);
        f.swap(free_);
    }
    if (!f.empty()) (void)hipDeviceSynchronize();
    for (auto& kv : f) (void)hipFree(kv.second);
}

int Buf::allocate(size_t bytes) {
    reset();
    if (bytes == 0) bytes = 256;
    p = Pool::get().alloc(bytes);
    if (!p) return fail(DLMA_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    n = bytes;
    return DLMA_OK;
}

// ---------------------------------------------------------------- gauge

int gauge_prepare(Gauge* g, int prec, hipStream_t s) {
    if (prec == P64 || g->lo_ready[prec]) return DLMA_OK;
    long nl = 2L * 4 * 9 * g->Vh, nc = 2L * 18 * g->Vh;
    size_t pb = pair_bytes(prec);
    if (prec == P16) {  // grouped layouts of the FP16 stencil (common.h)
        DLMA_TRY(g->Ulo[prec].allocate(nl * pb));
        DLMA_TRY(g->Cee[prec].allocate(2L * 20 * g->Vh * pb));
        DLMA_TRY(g->Cio[prec].allocate(2L * 20 * g->Vh * pb));
        DLMA_HIP(launch_regroup16(g->U64.as<double2>(), g->Ulo[prec].p, 8, 9, 3, g->Vh, s));
        DLMA_HIP(launch_regroup16(g->Cl64[0].as<double2>(), g->Cee[prec].p, 2, 18, 4, g->Vh, s));
        DLMA_HIP(launch_regroup16(g->Ci64.as<double2>(), g->Cio[prec].p, 2, 18, 4, g->Vh, s));
        g->lo_ready[prec] = true;
        return DLMA_OK;
    }
    DLMA_TRY(g->Ulo[prec].allocate(nl * pb));
    DLMA_TRY(g->Cee[prec].allocate(nc * pb));
    DLMA_TRY(g->Cio[prec].allocate(nc * pb));
    auto conv = [&](const void* src, void* dst, long n) -> hipError_t {
        switch (prec) {
        case P32: return launch_convert_pairs<P32>((const double2*)src, dst, n, s);
        case P16: return launch_convert_pairs<P16>((const double2*)src, dst, n, s);
        default: return launch_convert_pairs<PB16>((const double2*)src, dst, n, s);
        }
    };
    DLMA_HIP(conv(g->U64.p, g->Ulo[prec].p, nl));
    DLMA_HIP(conv(g->Cl64[0].p, g->Cee[prec].p, nc));
    DLMA_HIP(conv(g->Ci64.p, g->Cio[prec].p, nc));
    g->lo_ready[prec] = true;
    return DLMA_OK;
}

const void* gauge_links(const Gauge* g, int prec) { return prec == P64 ? g->U64.p : g->Ulo[prec].p; }
const void* gauge_clover_ee(const Gauge* g, int prec) { return prec == P64 ? g->Cl64[0].p : g->Cee[prec].p; }
const void* gauge_clover_oo_inv(const Gauge* g, int prec) { return prec == P64 ? g->Ci64.p : g->Cio[prec].p; }

// ---------------------------------------------------------------- tuning cache

static std::mutex g_tune_m;
static std::map<std::vector<int>, int> g_tuned;

int tuned_lookup(const int dims[4], int prec, int nrhs) {
    std::lock_guard<std::mutex> l(g_tune_m);
    auto it = g_tuned.find({dims[0], dims[1], dims[2], dims[3], prec, nrhs});
    return it == g_tuned.end() ? 0 : it->second;
}

void tuned_store(const int dims[4], int prec, int nrhs, int nb) {
    std::lock_guard<std::mutex> l(g_tune_m);
    g_tuned[{dims[0], dims[1], dims[2], dims[3], prec, nrhs}] = nb;
}

// ---------------------------------------------------------------- byte model

double hop_bytes(int prec, int kind, int flags, int Vh, int n) {
    double pb = (double)pair_bytes(prec);
    double sp = 12.0 * pb + (prec == P16 ? 4.0 : 0.0);  // one half-lattice spinor, per site
    double links = 8.0 * 9.0 * pb;                       // every link once per launch
    double clov = (kind == K2 && (flags & F_NOA)) ? 0.0 : 36.0 * pb;
    double vec;
    if (kind == K1) {
        vec = 2.0;                           // in, out
        if (flags & F_HASD) vec += 1.0;
        if (flags & F_ACCUM) vec += 1.0;
    } else {
        vec = 3.0;                           // in, x, out
        if (flags & F_HASB) vec += 1.0;
        if (flags & F_CG) vec = 6.0;         // in, x, r (r/w), xs (r/w)
    }
    // the shadow residual at the own site: one field shared by every RHS
    const double shared = (kind == K2 && (flags & (F_DOTR | F_DOTXH))) ? sp : 0.0;
    return (double)Vh * (links + clov + shared + vec * sp * n);
}

// ---------------------------------------------------------------- profiler

Profiler& Profiler::get() {
    static Profiler* p = new Profiler();
    return *p;
}

hipEvent_t Profiler::ev() {
    if (!spare.empty()) {
        hipEvent_t e = spare.back();
        spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

void Profiler::begin(int kc, double bytes, hipStream_t s, hipEvent_t& a) {
    (void)kc;
    (void)bytes;
    a = ev();
    (void)hipEventRecord(a, s);
}

void Profiler::end(hipEvent_t a, int kc, double bytes, hipStream_t s) {
    hipEvent_t b = ev();
    (void)hipEventRecord(b, s);
    pending.push_back({a, b, kc, bytes});
}

void Profiler::collect() {
    for (auto& p : pending) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
            launches[p.kc] += 1;
            ms[p.kc] += t;
            bytes[p.kc] += p.bytes;
        } else {
            (void)hipGetLastError();
        }
        spare.push_back(p.a);
        spare.push_back(p.b);
    }
    pending.clear();
}

}  // namespace dlma

extern "C" int dlma_release_cache(void) {
    dlma::Pool::get().trim();
    return DLMA_OK;
}
