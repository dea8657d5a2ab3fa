// C ABI: batched multi right-hand-side solver (dlma_solve) and the Schur-operator
// bandwidth benchmark (dlma_bench_schur).
//
// Structure of a solve (every launch covers all gauge sets and right-hand sides):
//   outer loop, FP64:   r = b - D x  (true residual, per-RHS norms)
//                       bhat_e = r_e - D_eo A_oo^-1 r_o
//   inner loop, prec P: CG on the normal equations Dhat Dhat^dag z = bhat_e with
//                       e = Dhat^dag z (CGNE), so the CG residual is the residual of
//                       Dhat e = bhat_e itself:
//                         w = Dhat^dag p; alpha = |r|^2/|w|^2; e += alpha w;
//                         r -= alpha Dhat w; beta = |r'|^2/|r|^2; p = r' + beta p
//   reconstruction:     x_e += e,  x_o += A_oo^-1 (r_o - D_oe e)
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "../../include/dlma.h"
#include "runtime.h"

using namespace dlma;

static inline hipStream_t S(void* s) { return (hipStream_t)s; }

extern "C" void dlma_solve_opts_default(dlma_solve_opts* o) {
    if (!o) return;
    o->tol = 1e-10;
    o->maxiter = 100000;
    o->max_outer = 40;
    o->prec = DLMA_PREC_FP64;
    o->inner_tol = 0.0;
    o->rhs_block = 0;
    o->use_x0 = 0;
    o->graph_iters = 8;
    o->check_every = 0;
    o->dagger = 0;
    o->lds_window = -1;
    o->inner_solver = 1;
}

namespace {

constexpr int MAXG = 16;

struct Cfg {
    Gauge* g;
    int nrhs, gidx;
    const double2* bcan;
    double2* xcan;
    Buf B, X, R, T, E;               // FP64: full B, X, R; half T (odd), E (even)
    Buf r, p, w, xs, y;              // inner vectors (precision P), half fields
    Buf nr, np, nw, nxs, ny;         // FP16 scales
    Buf part;                        // partial norms
    Buf tsup;                        // [nrhs][T] timeslice support of B (VecJob::tsup)
    Buf tdist;                       // [nrhs][T] distance to that support (in_reach), 0 after the first pass
    Buf parts;                       // BiCGStab, FP16: partials of (rh, s) from the s step
    Buf bs, bt, brh, nbs, nbt, nbrh;    // BiCGStab: s, t, shadow residual (precision P) and FP16 scales
    Buf bstate;                      // BiCGStab: rho alpha omega beta (complex, per rhs)
    double2 *brho = nullptr, *balpha = nullptr, *bomega = nullptr, *bbeta = nullptr;
    Buf dstate;                      // rr rr0 alpha beta tol2 abs2 nrm enrm (double) | active iters oact (int)
    int hnsb, vnsb;                  // site blocks of stencil and vector kernels
    double *rr, *rr0, *alpha, *beta, *tol2, *abs2, *nrm, *enrm;
    int *active, *iters;
    int* oact;  // right-hand sides iterated in the last pass: the FP64 outer stencils skip the others
    std::vector<double> bnorm2, rnorm2, relres;
    std::vector<int> used, conv, hact, hiters, hoact;
    std::vector<char> evenonly;      // rnorm2[r] holds the even sites' residual only
    int outer = 0;
};

template <int P> struct Tables {
    // device job tables
    Buf dresid, dprep, drecon, dresidE;        // HopJob<P64> (dresidE: the residual's even-site jobs)
    Buf dresidO, dprep0, drecon0;              // HopJob<P64>: odd-site residual; pass-0 jobs reading B as R
    Buf dvnB, dclov, dconv64, dacc64, dclov0;  // VecJob<P64>
    Buf dconv, dacc, dxpay;                    // VecJob<P>
    Buf dvnE, dfinE;                           // |E|^2 (Schur source) jobs
    Buf dvnE0, dconv640;                       // pass 0 from x = 0: the same, skipping where B vanishes
    Buf dk1d, dk2d, dk1, dk2cg;                // HopJob<P>
    Buf dfinB, dfinR, dfinI, dfinAB;           // FinJob
    int nresid = 0, nprep = 0, nrecon = 0, nvnB = 0, nclov = 0, nconv = 0, nk = 0, nfin = 0, nresidE = 0, bresidE = 0;
    int nresidO = 0, bresidO = 0;
    int bresid = 0, bprep = 0, brecon = 0, bvnB = 0, bclov = 0, bconv = 0, bxpay = 0, bvnE = 0;
    int bk1 = 0, bk2 = 0, bfin = 0;
    int nb64 = 1;                      // right-hand sides per thread of the FP64 outer stencils
    int wn = 0;                        // largest LDS window of the inner stencil jobs
    std::vector<FinJob> hfinI, hfinAB;  // kept for per-pass updates
    // BiCGStab: stencils p -> y -> v and s -> y -> t, the vector steps, the finishers
    bool bicg = false;
    Buf dbk1p, dbk2v, dbk1s, dbk2t, dbv, dbf;
    int nbv = 0, bbv = 0, bbf = 0;
    std::vector<BiFinJob> hbf;           // kept for per-pass updates (maxit)
};

template <class T> int upload(Buf& b, const std::vector<T>& v, hipStream_t s) {
    DLMA_TRY(b.allocate(sizeof(T) * std::max<size_t>(1, v.size())));
    if (!v.empty()) DLMA_HIP(hipMemcpyAsync(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
    return DLMA_OK;
}

template <int P> int alloc_cfg(Cfg& c, bool bicg, hipStream_t s) {
    Gauge* g = c.g;
    size_t n = c.nrhs;
    int Vh = g->Vh;
    size_t full64 = sizeof(double2) * n * 24 * Vh, half64 = sizeof(double2) * n * 12 * Vh;
    DLMA_TRY(c.B.allocate(full64));
    DLMA_TRY(c.X.allocate(full64));
    DLMA_TRY(c.tsup.allocate(sizeof(int) * (size_t)c.nrhs * g->geo.T));
    DLMA_TRY(c.tdist.allocate(sizeof(int) * (size_t)c.nrhs * g->geo.T));
    DLMA_TRY(c.R.allocate(full64));
    DLMA_TRY(c.T.allocate(half64));
    DLMA_TRY(c.E.allocate(half64));
    size_t halfP = pair_bytes(P) * n * 12 * Vh;
    DLMA_TRY(c.r.allocate(halfP));
    DLMA_TRY(c.p.allocate(halfP));
    DLMA_TRY(c.w.allocate(halfP));
    DLMA_TRY(c.xs.allocate(halfP));
    DLMA_TRY(c.y.allocate(halfP));
    if (P == P16) {
        size_t nb = sizeof(float) * n * Vh;
        DLMA_TRY(c.nr.allocate(nb));
        DLMA_TRY(c.np.allocate(nb));
        DLMA_TRY(c.nw.allocate(nb));
        DLMA_TRY(c.nxs.allocate(nb));
        DLMA_TRY(c.ny.allocate(nb));
    }
    if (bicg) {
        DLMA_TRY(c.bs.allocate(halfP));
        DLMA_TRY(c.bt.allocate(halfP));
        DLMA_TRY(c.brh.allocate(pair_bytes(P) * 12 * Vh));  // one shadow residual, shared by every RHS
        if (P == P16) {
            size_t nb = sizeof(float) * n * Vh;
            DLMA_TRY(c.nbs.allocate(nb));
            DLMA_TRY(c.nbt.allocate(nb));
            DLMA_TRY(c.nbrh.allocate(sizeof(float) * Vh));
        }
        DLMA_TRY(c.bstate.allocate(sizeof(double2) * 4 * n));
        c.brho = c.bstate.as<double2>();
        c.balpha = c.brho + n;
        c.bomega = c.brho + 2 * n;
        c.bbeta = c.brho + 3 * n;
        DLMA_HIP(hipMemsetAsync(c.bstate.p, 0, sizeof(double2) * 4 * n, s));
    }
    c.hnsb = hop_nsb(g->geo);
    c.vnsb = ceil_div(Vh, VEC_BS);
    int pmax = std::max(std::max(2 * c.hnsb, 3 * c.vnsb), hop_nq(F_DOTX | F_DOTXH) * c.hnsb);
    DLMA_TRY(c.part.allocate(sizeof(double) * n * pmax));
    if (bicg) DLMA_TRY(c.parts.allocate(sizeof(double) * n * 2 * c.vnsb));
    DLMA_TRY(c.dstate.allocate(sizeof(double) * 8 * n + sizeof(int) * 3 * n + 256));
    double* d = c.dstate.as<double>();
    c.rr = d; c.rr0 = d + n; c.alpha = d + 2 * n; c.beta = d + 3 * n; c.tol2 = d + 4 * n; c.abs2 = d + 5 * n;
    c.nrm = d + 6 * n;
    c.enrm = d + 7 * n;
    c.active = (int*)(d + 8 * n);
    c.iters = c.active + n;
    c.oact = c.iters + n;
    DLMA_HIP(hipMemsetAsync(c.dstate.p, 0, sizeof(double) * 8 * n + sizeof(int) * 3 * n, s));
    c.bnorm2.assign(n, 0); c.rnorm2.assign(n, 0); c.relres.assign(n, 0);
    c.used.assign(n, 0); c.conv.assign(n, 0); c.hact.assign(n, 0); c.hiters.assign(n, 0); c.hoact.assign(n, 1);
    c.evenonly.assign(n, 0);
    return DLMA_OK;
}

template <int P> float* nrm_of(const Buf& b) { return P == P16 ? b.as<float>() : nullptr; }

template <int P> int build_tables(std::vector<Cfg>& cs, Tables<P>& t, int nb, int sg_in, int win, int nb64, int sg64, hipStream_t s) {
    std::vector<HopJob<P64>> resid, prep, recon, residE, residO, prep0, recon0;
    std::vector<VecJob<P64>> vnB, clov, conv64, acc64, vnE, clov0, vnE0, conv640;
    std::vector<VecJob<P>> conv, acc, xpay;
    std::vector<HopJob<P>> k1d, k2d, k1, k2cg, bk1p, bk2v, bk1s, bk2t;
    std::vector<FinJob> finB, finR, finI, finAB, finE;
    std::vector<BiVecJob<P>> bvv;
    std::vector<BiFinJob> bfv;
    int rhs0B = 0, rhs0R = 0, rhs0I = 0, rhs0AB = 0, rhs0E = 0, rhs0BF = 0;
    for (auto& c : cs) {
        Gauge* g = c.g;
        int Vh = g->Vh, n = c.nrhs;
        const double2* U64 = g->U64.as<double2>();
        int* tsup = c.tsup.as<int>();
        const int vt = g->geo.Z * g->geo.Y * g->geo.Xh, T = g->geo.T;
        // the support flags of B on a vector job; dil: the job's input vanishes where
        // t - dil .. t + dil are unflagged
        auto with_support = [&](VecJob<P64> v, int dil) {
            v.tsup = tsup; v.tdil = dil; v.vt = vt; v.T = T;
            return v;
        };
        for (int par = 0; par < 2; ++par) {
            HopJob<P64> j = hop_job<P64>(g, par, n, nb64);
            j.sg = sg64;
            j.U = U64;
            j.C = g->Cl64[par].as<double2>();
            j.b = full_view(c.B.p, Vh, par);
            j.tsup = tsup;  // b is read where B is nonzero only
            j.x = full_view(c.X.p, Vh, par);
            j.in = full_view(c.X.p, Vh, 1 - par);
            j.out = full_view(c.R.p, Vh, par);
            j.part = c.part.as<double>() + (size_t)par * c.hnsb;
            j.pstride = 2 * c.hnsb;
            j.cb = 1.0; j.ca = -1.0; j.ch = 0.5;
            if (par == 1) residO.push_back(j);  // the final check covers every right-hand side
            j.active = c.oact;  // converged right-hand sides keep their last residual
            resid.push_back(j);
            if (par == 0) {  // with R_o = 0 the even residual is the Schur source E itself
                HopJob<P64> je = j;
                je.out = half_view<P64>(c.E.p, nullptr, Vh);
                if (P == P16) {  // x_e += e of the last inner solve, fused (F_ACCX)
                    je.in16 = half_view<P16>(c.xs.p, nrm_of<P16>(c.nxs), Vh);
                    je.in16s = c.enrm;
                }
                residE.push_back(je);
            }
            VecJob<P64> v = {};
            v.Vh = Vh; v.nrhs = n; v.nsb = c.vnsb;
            v.a = full_view(c.B.p, Vh, par);
            v.part = c.part.as<double>() + (size_t)par * c.vnsb;
            v.pstride = 2 * c.vnsb;
            v.tsup_out = tsup;  // |B|^2 also records where B is nonzero
            v.vt = vt; v.T = T;
            vnB.push_back(v);
        }
        {   // T = A_oo^-1 R_o
            VecJob<P64> v = {};
            v.Vh = Vh; v.nrhs = n; v.nsb = c.vnsb;
            v.a = full_view(c.R.p, Vh, 1);
            v.c = half_view<P64>(c.T.p, nullptr, Vh);
            v.C = g->Ci64.as<double2>();
            clov.push_back(v);
            v.a = full_view(c.B.p, Vh, 1);  // first pass from x = 0: R = B
            clov0.push_back(with_support(v, 0));
        }
        {   // E = R_e + 1/2 H T
            HopJob<P64> j = hop_job<P64>(g, 0, n, nb64);
            j.sg = sg64;
            j.U = U64;
            j.x = full_view(c.R.p, Vh, 0);
            j.in = half_view<P64>(c.T.p, nullptr, Vh);
            j.out = half_view<P64>(c.E.p, nullptr, Vh);
            j.ca = 1.0; j.ch = 0.5;
            prep.push_back(j);
            j.x = full_view(c.B.p, Vh, 0);
            j.tsup = tsup;  // E = 0 where B vanishes on t - 1 .. t + 1
            prep0.push_back(j);
        }
        {   // r = p = P(E), xs = 0 ; and accumulate E = xs, X_e += E
            VecJob<P> v = {};
            v.Vh = Vh; v.nrhs = n; v.nsb = c.vnsb;
            v.a = half_view<P>(c.r.p, nrm_of<P>(c.nr), Vh);
            v.b = half_view<P>(c.p.p, nrm_of<P>(c.np), Vh);
            v.c = half_view<P>(c.xs.p, nrm_of<P>(c.nxs), Vh);
            v.part = c.part.as<double>();
            v.pstride = c.vnsb;
            v.s = c.enrm;
            v.active = c.oact;  // the others keep r, p, xs (xs is not added to x for them)
            conv.push_back(v);
            VecJob<P64> v64 = {};
            v64.Vh = Vh; v64.nrhs = n; v64.nsb = c.vnsb;
            v64.a = half_view<P64>(c.E.p, nullptr, Vh);
            conv64.push_back(v64);
            conv640.push_back(with_support(v64, 1));
            VecJob<P64> e64 = v64;
            e64.part = c.part.as<double>();
            e64.pstride = c.vnsb;
            vnE.push_back(e64);
            vnE0.push_back(with_support(e64, 1));
            VecJob<P> a = v;
            a.a = half_view<P>(c.xs.p, nrm_of<P>(c.nxs), Vh);
            acc.push_back(a);
            VecJob<P64> a64 = v64;
            a64.b = full_view(c.X.p, Vh, 0);
            if (P == P16) a64.a.v = nullptr;  // the reconstruction reads the FP16 solution
            acc64.push_back(a64);
            VecJob<P> x = v;
            x.a = half_view<P>(c.r.p, nrm_of<P>(c.nr), Vh);
            x.b = half_view<P>(c.p.p, nrm_of<P>(c.np), Vh);
            x.s = c.beta;
            x.active = c.active;
            xpay.push_back(x);
        }
        {   // X_o += A_oo^-1 (R_o + 1/2 H E)
            HopJob<P64> j = hop_job<P64>(g, 1, n, nb64);
            j.sg = sg64;
            j.U = U64;
            j.C = g->Ci64.as<double2>();
            j.in = half_view<P64>(c.E.p, nullptr, Vh);
            if (P == P16) {  // E as the FP16 solution times |bhat|: 4 loads per site, not 12
                j.in16 = half_view<P16>(c.xs.p, nrm_of<P16>(c.nxs), Vh);
                j.in16s = c.enrm;
            }
            j.x = full_view(c.R.p, Vh, 1);
            j.out = full_view(c.X.p, Vh, 1);
            j.ch = 0.5;
            j.active = c.oact;  // E = 0 for the others
            recon.push_back(j);
            j.x = full_view(c.B.p, Vh, 1);
            j.tsup = tsup;  // d = B_o is read where B is nonzero only
            recon0.push_back(j);
        }
        {   // inner CG stencils
            const typename PT<P>::S* U = (const typename PT<P>::S*)gauge_links(g, P);
            const typename PT<P>::S* Cee = (const typename PT<P>::S*)gauge_clover_ee(g, P);
            const typename PT<P>::S* Cio = (const typename PT<P>::S*)gauge_clover_oo_inv(g, P);
            SF<P> vp = half_view<P>(c.p.p, nrm_of<P>(c.np), Vh), vy = half_view<P>(c.y.p, nrm_of<P>(c.ny), Vh);
            SF<P> vw = half_view<P>(c.w.p, nrm_of<P>(c.nw), Vh), vr = half_view<P>(c.r.p, nrm_of<P>(c.nr), Vh);
            SF<P> vx = half_view<P>(c.xs.p, nrm_of<P>(c.nxs), Vh);
            HopJob<P> j1 = hop_job<P>(g, 1, n, nb, win != 0);
            j1.U = U; j1.C = Cio; j1.ch = -0.5; j1.active = c.active; j1.sg = sg_in;
            HopJob<P> j2 = hop_job<P>(g, 0, n, nb, win != 0);
            j2.U = U; j2.C = Cee; j2.ca = 1.0; j2.ch = 0.5; j2.active = c.active; j2.sg = sg_in;
            j2.part = c.part.as<double>(); j2.pstride = c.hnsb;
            HopJob<P> a = j1; a.in = vp; a.out = vy; k1d.push_back(a);
            HopJob<P> b = j2; b.x = vp; b.in = vy; b.out = vw; k2d.push_back(b);
            HopJob<P> d = j1; d.in = vw; d.out = vy; k1.push_back(d);
            HopJob<P> e = j2; e.x = vw; e.in = vy; e.r = vr; e.xs = vx; e.alpha = c.alpha; k2cg.push_back(e);
            t.wn = std::max(t.wn, std::max(j1.wn, j2.wn));
            if (t.bicg) {  // BiCGStab: v = w's storage, x = xs's
                SF<P> vs = half_view<P>(c.bs.p, nrm_of<P>(c.nbs), Vh), vt = half_view<P>(c.bt.p, nrm_of<P>(c.nbt), Vh);
                SF<P> vrh = half_view<P>(c.brh.p, nrm_of<P>(c.nbrh), Vh);
                vrh.rs = 0;  // every RHS reads the one shadow residual
                vrh.ns = 0;
                HopJob<P> k1 = j1; k1.part = nullptr;
                HopJob<P> k2 = j2;  // partials of (rh, v), then of (t, s) and |t|^2 (hop_nq layout)
                HopJob<P> a1 = k1; a1.in = vp; a1.out = vy; bk1p.push_back(a1);
                HopJob<P> a2 = k2; a2.x = vp; a2.in = vy; a2.out = vw; a2.r = vrh; bk2v.push_back(a2);
                HopJob<P> a3 = k1; a3.in = vs; a3.out = vy; bk1s.push_back(a3);
                HopJob<P> a4 = k2; a4.x = vs; a4.in = vy; a4.out = vt; a4.r = vrh; bk2t.push_back(a4);
                BiVecJob<P> bv = {};
                bv.Vh = Vh; bv.nrhs = n; bv.nsb = c.vnsb;
                bv.r = vr; bv.rh = vrh; bv.p = vp; bv.v = vw; bv.s = vs; bv.t = vt; bv.x = vx;
                bv.alpha = c.balpha; bv.omega = c.bomega; bv.beta = c.bbeta;
                bv.active = c.active; bv.part = c.part.as<double>(); bv.pstride = c.vnsb;
                bv.part_s = c.parts.as<double>();
                if (P == P16) {
                    bv.tdist = c.tdist.as<int>();
                    bv.titer = c.iters;
                    bv.vt = g->geo.Z * g->geo.Y * g->geo.Xh;
                    bv.T = g->geo.T;
                }
                bvv.push_back(bv);
                BiFinJob bf = {};
                bf.nrhs = n; bf.rhs0 = rhs0BF; rhs0BF += n; bf.npart = c.vnsb; bf.nparth = c.hnsb;
                bf.part = c.part.as<double>();
                bf.part_s = c.parts.as<double>();
                bf.rho = c.brho; bf.alpha = c.balpha; bf.omega = c.bomega; bf.beta = c.bbeta;
                bf.rr = c.rr; bf.tol2 = c.tol2; bf.active = c.active; bf.iters = c.iters; bf.maxit = 1 << 30;
                bfv.push_back(bf);
            }
        }
        FinJob f = {};
        f.nrhs = n; f.part = c.part.as<double>();
        f.rr = c.rr; f.rr0 = c.rr0; f.alpha = c.alpha; f.beta = c.beta; f.tol2 = c.tol2; f.abs2 = c.abs2;
        f.active = c.active; f.iters = c.iters; f.out = c.nrm; f.maxit = 1 << 30;
        FinJob fb = f; fb.npart = 2 * c.vnsb; fb.rhs0 = rhs0B; rhs0B += n; finB.push_back(fb);
        FinJob fr = f; fr.npart = 2 * c.hnsb; fr.rhs0 = rhs0R; rhs0R += n; finR.push_back(fr);
        FinJob fi = f; fi.npart = c.vnsb; fi.rhs0 = rhs0I; rhs0I += n; fi.out = c.enrm; finI.push_back(fi);
        FinJob fe = f; fe.npart = c.vnsb; fe.rhs0 = rhs0E; rhs0E += n; fe.out = c.enrm; finE.push_back(fe);
        FinJob fa = f; fa.npart = c.hnsb; fa.rhs0 = rhs0AB; rhs0AB += n; finAB.push_back(fa);
    }
    t.bresid = assign_blocks(resid); t.bprep = assign_blocks(prep); t.brecon = assign_blocks(recon);
    t.bresidE = assign_blocks(residE);
    t.nresidE = (int)residE.size();
    DLMA_TRY(upload(t.dresidE, residE, s));
    t.bresidO = assign_blocks(residO);
    t.nresidO = (int)residO.size();
    DLMA_TRY(upload(t.dresidO, residO, s));
    assign_blocks(prep0); assign_blocks(recon0); assign_vec_blocks(clov0);
    DLMA_TRY(upload(t.dprep0, prep0, s)); DLMA_TRY(upload(t.drecon0, recon0, s)); DLMA_TRY(upload(t.dclov0, clov0, s));
    t.bvnB = assign_vec_blocks(vnB); t.bclov = assign_vec_blocks(clov);
    t.bconv = assign_vec_blocks(conv); assign_vec_blocks(conv64); assign_vec_blocks(acc); assign_vec_blocks(acc64);
    t.bvnE = assign_vec_blocks(vnE);
    assign_vec_blocks(vnE0); assign_vec_blocks(conv640);
    DLMA_TRY(upload(t.dvnE0, vnE0, s)); DLMA_TRY(upload(t.dconv640, conv640, s));
    t.bxpay = assign_vec_blocks(xpay);
    t.bk1 = assign_blocks(k1d); assign_blocks(k1);
    t.bk2 = assign_blocks(k2d); assign_blocks(k2cg);
    t.bfin = rhs0AB;
    if (t.bicg) {
        assign_blocks(bk1p); assign_blocks(bk2v); assign_blocks(bk1s); assign_blocks(bk2t);
        int b = 0;
        for (auto& v : bvv) { v.blk0 = b; b += v.nsb * v.nrhs; }
        t.bbv = b;
        t.nbv = (int)bvv.size();
        t.bbf = rhs0BF;
        t.hbf = bfv;
        DLMA_TRY(upload(t.dbk1p, bk1p, s)); DLMA_TRY(upload(t.dbk2v, bk2v, s));
        DLMA_TRY(upload(t.dbk1s, bk1s, s)); DLMA_TRY(upload(t.dbk2t, bk2t, s));
        DLMA_TRY(upload(t.dbv, bvv, s)); DLMA_TRY(upload(t.dbf, bfv, s));
    }
    t.nb64 = nb64;
    t.nresid = (int)resid.size(); t.nprep = (int)prep.size(); t.nrecon = (int)recon.size();
    t.nvnB = (int)vnB.size(); t.nclov = (int)clov.size(); t.nconv = (int)conv.size(); t.nk = (int)k1d.size();
    t.nfin = (int)finAB.size();
    DLMA_TRY(upload(t.dresid, resid, s)); DLMA_TRY(upload(t.dprep, prep, s)); DLMA_TRY(upload(t.drecon, recon, s));
    DLMA_TRY(upload(t.dvnB, vnB, s)); DLMA_TRY(upload(t.dclov, clov, s)); DLMA_TRY(upload(t.dconv64, conv64, s));
    DLMA_TRY(upload(t.dacc64, acc64, s)); DLMA_TRY(upload(t.dconv, conv, s)); DLMA_TRY(upload(t.dacc, acc, s));
    DLMA_TRY(upload(t.dxpay, xpay, s));
    DLMA_TRY(upload(t.dvnE, vnE, s));
    DLMA_TRY(upload(t.dfinE, finE, s));
    DLMA_TRY(upload(t.dk1d, k1d, s)); DLMA_TRY(upload(t.dk2d, k2d, s)); DLMA_TRY(upload(t.dk1, k1, s));
    DLMA_TRY(upload(t.dk2cg, k2cg, s));
    DLMA_TRY(upload(t.dfinB, finB, s)); DLMA_TRY(upload(t.dfinR, finR, s));
    t.hfinI = finI;
    t.hfinAB = finAB;
    DLMA_TRY(upload(t.dfinI, finI, s)); DLMA_TRY(upload(t.dfinAB, finAB, s));
    DLMA_HIP(hipStreamSynchronize(s));  // host job vectors go out of scope
    return DLMA_OK;
}

// one timed stencil launch (events bracket it while profiling is on)
template <int P> int hop_launch(const HopCfg& hc, const void* djobs, int njob, int nblk, int kc, double bytes, hipStream_t s) {
    Profiler& pr = Profiler::get();
    hipEvent_t a = nullptr;
    if (pr.on) pr.begin(kc, bytes, s, a);
    DLMA_HIP(launch_hop<P>(hc, (const HopJob<P>*)djobs, njob, nblk, s));
    if (pr.on) pr.end(a, kc, bytes, s);
    return DLMA_OK;
}

// DLMA_LOG=2: after each launch of the inner iteration, count non-finite entries of the
// vector it wrote (first configuration), to locate where a breakdown starts.
template <int P> int debug_field(Cfg& c, const Buf& v, const Buf& nv, const char* what, hipStream_t s) {
    Buf o;
    DLMA_TRY(o.allocate(sizeof(double) * 4));
    double init[4] = {0, 0, 1e300, 1e300};
    DLMA_HIP(hipMemcpyAsync(o.p, init, sizeof(init), hipMemcpyHostToDevice, s));
    DLMA_HIP(launch_check_field<P>(half_view<P>(v.p, nrm_of<P>(nv), c.g->Vh), c.g->Vh, c.nrhs, o.as<double>(), s));
    double h[4];
    DLMA_HIP(hipMemcpyAsync(h, o.p, sizeof(h), hipMemcpyDeviceToHost, s));
    DLMA_HIP(hipStreamSynchronize(s));
    std::fprintf(stderr, "[dlma]     %-3s non-finite %.0f, denormal-max sites %.0f, min site max %.3e, min scale %.3e\n", what,
                 h[0], h[1], h[2], h[3]);
    return DLMA_OK;
}

template <int P> int cg_iteration(std::vector<Cfg>& cs, Tables<P>& t, int nb, const std::vector<int>& nact, hipStream_t s) {
    static const bool dbg = std::getenv("DLMA_LOG") && std::getenv("DLMA_LOG")[0] == '2';
    double b1 = 0, b2 = 0, b3 = 0;
    if (Profiler::get().on)
        for (size_t i = 0; i < cs.size(); ++i) {
            b1 += hop_bytes(P, K1, F_G5IN, cs[i].g->Vh, nact[i]);
            b2 += hop_bytes(P, K2, F_G5OUT | F_NORM, cs[i].g->Vh, nact[i]);
            b3 += hop_bytes(P, K2, F_CG, cs[i].g->Vh, nact[i]);
        }
    Cfg& c0 = cs[0];
    if (dbg) DLMA_TRY(debug_field<P>(c0, c0.p, c0.np, "p", s));
    DLMA_TRY(hop_launch<P>(HopCfg{K1, F_G5IN, nb, t.wn}, t.dk1d.p, t.nk, t.bk1, KC_K1DAG, b1, s));
    if (dbg) DLMA_TRY(debug_field<P>(c0, c0.y, c0.ny, "y1", s));
    DLMA_TRY(hop_launch<P>(HopCfg{K2, F_G5OUT | F_NORM, nb, t.wn}, t.dk2d.p, t.nk, t.bk2, KC_K2DAGN, b2, s));
    if (dbg) DLMA_TRY(debug_field<P>(c0, c0.w, c0.nw, "w", s));
    DLMA_HIP(launch_finish(t.dfinAB.template as<FinJob>(), t.nfin, t.bfin, FIN_ALPHA, s));
    DLMA_TRY(hop_launch<P>(HopCfg{K1, 0, nb, t.wn}, t.dk1.p, t.nk, t.bk1, KC_K1, b1, s));
    if (dbg) DLMA_TRY(debug_field<P>(c0, c0.y, c0.ny, "y2", s));
    DLMA_TRY(hop_launch<P>(HopCfg{K2, F_CG, nb, t.wn}, t.dk2cg.p, t.nk, t.bk2, KC_K2CG, b3, s));
    if (dbg) DLMA_TRY(debug_field<P>(c0, c0.r, c0.nr, "r", s));
    if (dbg) DLMA_TRY(debug_field<P>(c0, c0.xs, c0.nxs, "xs", s));
    DLMA_HIP(launch_finish(t.dfinAB.template as<FinJob>(), t.nfin, t.bfin, FIN_BETA, s));
    DLMA_HIP(launch_xpay<P>(t.dxpay.template as<VecJob<P>>(), t.nconv, t.bxpay, s));
    return DLMA_OK;
}

// One BiCGStab iteration on Dhat for every configuration (the steps of bicg.hip with
// the solver's stencil kernels for the two operator applications).
// FP16 fields take the merged iteration: K2 for t also forms (rh, t) of the stored t
// and the s step (rh, s) of the stored s, so rho' = (rh, s) - omega (rh, t) and beta
// are known before the updates, and x, r and p are updated in one pass (9 launches,
// 11 field passes of the vector steps instead of 13).  The other precisions run the
// three separate updates.
constexpr int bicg_dotx_flags(int P) { return P == P16 ? (F_DOTX | F_DOTXH) : F_DOTX; }

// Timeslice windows of the four stencil launches of one iteration (K1 of p, K2 for v,
// K1 of s, K2 for t; twn = 0: every timeslice).  Used by the first pass of a single
// configuration while its Krylov vectors have not reached every timeslice.
struct IterWin { int tw0[4], twn[4]; };

template <int P>
int bicg_iteration(std::vector<Cfg>& cs, Tables<P>& t, int nb, const std::vector<int>& nact, hipStream_t s,
                   const IterWin* w = nullptr) {
    constexpr int FX = bicg_dotx_flags(P);
    double b1 = 0, b2v = 0, b2t = 0;
    if (Profiler::get().on)
        for (size_t i = 0; i < cs.size(); ++i) {
            b1 += hop_bytes(P, K1, 0, cs[i].g->Vh, nact[i]);
            b2v += hop_bytes(P, K2, F_DOTR, cs[i].g->Vh, nact[i]);
            b2t += hop_bytes(P, K2, FX, cs[i].g->Vh, nact[i]);
        }
    const BiVecJob<P>* bv = t.dbv.template as<BiVecJob<P>>();
    const BiFinJob* bf = t.dbf.template as<BiFinJob>();
    // a windowed launch covers fewer blocks (and bytes); a windowed K2 leaves the partial
    // sums of the other site blocks unwritten, so they are cleared first
    auto launch = [&](int i, int kind, int flags, const Buf& jobs, int nblk, int kc, double bytes) -> int {
        HopCfg hc{kind, flags, nb, t.wn};
        if (w && w->twn[i] > 0) {
            Cfg& c = cs[0];
            const int T = c.g->geo.T;
            hc.tw0 = w->tw0[i];
            hc.twn = w->twn[i];
            nblk = hop_window_blocks(c.g->geo, c.nrhs, nb, w->twn[i]);
            bytes *= (double)w->twn[i] / T;
            if (hop_nq(flags) > 0)
                DLMA_HIP(hipMemsetAsync(c.part.p, 0, sizeof(double) * (size_t)c.nrhs * hop_nq(flags) * c.hnsb, s));
        }
        return hop_launch<P>(hc, jobs.p, t.nk, nblk, kc, bytes, s);
    };
    DLMA_TRY(launch(0, K1, 0, t.dbk1p, t.bk1, KC_K1, b1));
    DLMA_TRY(launch(1, K2, F_DOTR, t.dbk2v, t.bk2, KC_K2V, b2v));
    DLMA_HIP(launch_bifinish(bf, t.nbv, t.bbf, BF_ALPHA, s));
    DLMA_HIP(launch_bivec<P>(bv, t.nbv, t.bbv, P == P16 ? BV_SH : BV_S, s));
    DLMA_TRY(launch(2, K1, 0, t.dbk1s, t.bk1, KC_K1, b1));
    DLMA_TRY(launch(3, K2, FX, t.dbk2t, t.bk2, KC_K2T, b2t));
    if (P == P16) {
        DLMA_HIP(launch_bifinish(bf, t.nbv, t.bbf, BF_OMBETA, s));
        DLMA_HIP(launch_bivec<P>(bv, t.nbv, t.bbv, BV_XRP, s));
        DLMA_HIP(launch_bifinish(bf, t.nbv, t.bbf, BF_CONV, s));
        return DLMA_OK;
    }
    DLMA_HIP(launch_bifinish(bf, t.nbv, t.bbf, BF_OMEGA, s));
    DLMA_HIP(launch_bivec<P>(bv, t.nbv, t.bbv, BV_XR, s));
    DLMA_HIP(launch_bifinish(bf, t.nbv, t.bbf, BF_BETA, s));
    DLMA_HIP(launch_bivec<P>(bv, t.nbv, t.bbv, BV_P, s));
    return DLMA_OK;
}

template <int P> int inner_iteration(std::vector<Cfg>& cs, Tables<P>& t, int nb, const std::vector<int>& nact, hipStream_t s) {
    return t.bicg ? bicg_iteration<P>(cs, t, nb, nact, s) : cg_iteration<P>(cs, t, nb, nact, s);
}

// The inner iterations as one HIP graph: `iters` consecutive CG iterations are
// captured once per solve on a library stream and replayed with one launch.  Every
// parameter the kernels read lives in device memory (job tables, per-RHS scalars,
// active flags), so the captured launches stay valid for the whole solve.  The
// iteration contains kernel launches only (no memset or copy nodes).
struct IterGraph {
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    IterGraph() = default;
    IterGraph(const IterGraph&) = delete;
    IterGraph& operator=(const IterGraph&) = delete;
    ~IterGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

template <int P>
int capture_iterations(std::vector<Cfg>& cs, Tables<P>& t, int nb, const std::vector<int>& nact, int iters, IterGraph& ig) {
    DLMA_HIP(hipStreamCreateWithFlags(&ig.cap, hipStreamNonBlocking));
    DLMA_HIP(hipStreamBeginCapture(ig.cap, hipStreamCaptureModeRelaxed));
    int rc = DLMA_OK;
    for (int k = 0; k < iters && rc == DLMA_OK; ++k) rc = inner_iteration<P>(cs, t, nb, nact, ig.cap);
    hipError_t e = hipStreamEndCapture(ig.cap, &ig.graph);
    if (rc != DLMA_OK) return rc;
    if (e != hipSuccess) return fail(DLMA_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    DLMA_HIP(hipGraphInstantiate(&ig.exec, ig.graph, nullptr, nullptr, 0));
    return DLMA_OK;
}

struct Tune { int nb, sg, win; };  // win: FP16 stencils stage their LDS window
template <int P> int tune_hop(Gauge* g, int nrhs, int fixed_nb, SF<P> vp, SF<P> vy, SF<P> vw, Tune& out, hipStream_t s);

template <int P>
int solve_impl(std::vector<Cfg>& cs, const dlma_solve_opts& o, hipStream_t s) {
    for (auto& c : cs) {
        DLMA_TRY(gauge_prepare(c.g, P, s));
        DLMA_TRY(alloc_cfg<P>(c, o.inner_solver == 1, s));
    }
    if (o.rhs_block < 0 || o.rhs_block > 4)
        return fail(DLMA_EINVAL, "rhs_block must be 0 .. 4");
    // launch shapes, tuned on the largest configuration: inner stencils (precision P) and
    // the FP64 outer stencils (one right-hand side per thread)
    size_t big = 0;
    for (size_t i = 1; i < cs.size(); ++i)
        if ((long)cs[i].g->Vh * cs[i].nrhs > (long)cs[big].g->Vh * cs[big].nrhs) big = i;
    Tune tin{1, 0, 1}, t64{1, 0, 0};
    {
        Cfg& c = cs[big];
        int Vh = c.g->Vh;
        DLMA_TRY(tune_hop<P>(c.g, c.nrhs, o.rhs_block, half_view<P>(c.p.p, nrm_of<P>(c.np), Vh),
                             half_view<P>(c.y.p, nrm_of<P>(c.ny), Vh), half_view<P>(c.w.p, nrm_of<P>(c.nw), Vh), tin, s));
        DLMA_TRY(tune_hop<P64>(c.g, c.nrhs, 0, half_view<P64>(c.E.p, nullptr, Vh), half_view<P64>(c.T.p, nullptr, Vh),
                               full_view(c.R.p, Vh, 0), t64, s));
    }
    if (o.lds_window >= 0) tin.win = o.lds_window;
    const int nb = tin.nb;
    Tables<P> t;
    t.bicg = o.inner_solver == 1;
    if (t.bicg)  // BiCGStab's shadow residual: one fixed seeded random field per configuration
        for (auto& c : cs)
            DLMA_HIP(launch_fill_random<P>(half_view<P>(c.brh.p, nrm_of<P>(c.nbrh), c.g->Vh), c.g->Vh, 1,
                                           0x5eedu + (unsigned)c.gidx, s));
    DLMA_TRY(build_tables<P>(cs, t, nb, tin.sg, tin.win, t64.nb, t64.sg, s));
    int ncfg = (int)cs.size();
    // load sources and start vectors
    for (auto& c : cs) {
        // D^dag x = b  <=>  D (g5 x) = g5 b: solve for X = g5 x with source g5 b
        DLMA_HIP(launch_canon_to_eo(c.bcan, c.B.as<double2>(), c.g->geo, c.nrhs, s, o.dagger));
        if (o.use_x0) DLMA_HIP(launch_canon_to_eo(c.xcan, c.X.as<double2>(), c.g->geo, c.nrhs, s, o.dagger));
        else DLMA_HIP(hipMemsetAsync(c.X.p, 0, c.X.n, s));
        DLMA_HIP(hipMemsetAsync(c.tsup.p, 0, c.tsup.n, s));  // set by the norm of B
    }
    DLMA_HIP(launch_norm<P64>(t.dvnB.template as<VecJob<P64>>(), t.nvnB, t.bvnB, s));
    // first pass from x = 0 (FP16 BiCGStab): distances to each source's support, for the
    // reach of the Krylov vectors; otherwise 0 (everything within reach)
    const bool reach_skip = P == P16 && t.bicg && !o.use_x0;
    for (auto& c : cs) {
        if (reach_skip) DLMA_HIP(launch_tdist(c.tsup.as<int>(), c.tdist.as<int>(), c.nrhs, c.g->geo.T, s));
        else DLMA_HIP(hipMemsetAsync(c.tdist.p, 0, c.tdist.n, s));
    }
    DLMA_HIP(launch_finish(t.dfinB.template as<FinJob>(), t.nfin, t.bfin, FIN_NORM, s));
    for (auto& c : cs) DLMA_HIP(hipMemcpyAsync(c.bnorm2.data(), c.nrm, sizeof(double) * c.nrhs, hipMemcpyDeviceToHost, s));
    // One configuration: the shortest periodic arc [arc0, arc0 + arcn) of timeslices that
    // holds every source's support.  While the first pass's Krylov vectors have not left
    // its neighbourhood, its stencils launch over that neighbourhood only (IterWin).
    std::vector<int> hsup;
    if (reach_skip && cs.size() == 1) {
        hsup.resize((size_t)cs[0].nrhs * cs[0].g->geo.T);
        DLMA_HIP(hipMemcpyAsync(hsup.data(), cs[0].tsup.p, sizeof(int) * hsup.size(), hipMemcpyDeviceToHost, s));
    }
    DLMA_HIP(hipStreamSynchronize(s));
    int arc0 = 0, arcn = 0;
    if (!hsup.empty()) {
        const int T = cs[0].g->geo.T;
        std::vector<char> any(T, 0);
        for (int r = 0; r < cs[0].nrhs; ++r)
            for (int tt = 0; tt < T; ++tt) any[tt] |= hsup[(size_t)r * T + tt] != 0;
        // the longest run of empty timeslices (periodic); the arc is the rest
        int best = -1, bstart = 0;
        for (int tt = 0; tt < T; ++tt) {
            if (any[tt] || any[(tt + T - 1) % T] == 0) continue;  // runs start after a flagged timeslice
            int len = 0;
            while (len < T && !any[(tt + len) % T]) ++len;
            if (len > best) { best = len; bstart = tt; }
        }
        if (best > 0) {  // otherwise every timeslice holds a source (or none does)
            arc0 = (bstart + best) % T;
            arcn = T - best;
        }
    }
    bool nan = false;
    for (auto& c : cs) {
        std::vector<double> abs2(c.nrhs);
        for (int r = 0; r < c.nrhs; ++r) {
            if (!std::isfinite(c.bnorm2[r])) nan = true;
            abs2[r] = 0.25 * o.tol * o.tol * c.bnorm2[r];
        }
        DLMA_HIP(hipMemcpyAsync(c.abs2, abs2.data(), sizeof(double) * c.nrhs, hipMemcpyHostToDevice, s));
        DLMA_HIP(hipStreamSynchronize(s));
    }
    if (nan) return fail(DLMA_ENAN, "non-finite value in a source");
    static const bool dlog = std::getenv("DLMA_LOG") != nullptr;
    // Per-pass reduction of the inner residual.  FP16: the true residual drops 2-7 times
    // less per pass than the inner one (storage rounding), so 1e-3 brings every right-hand
    // side of a 192-RHS batch below 1e-10 in four passes with a factor of two to spare;
    // looser values take as long in total, with a fifth pass for the stragglers.
    double rel = o.inner_tol > 0 ? o.inner_tol : (P == P64 ? 0.0 : (P == P32 ? 1e-5 : (P == P16 ? 1e-3 : 1e-2)));
    int check = o.check_every > 0 ? o.check_every : 8;
    // hipGraph replay of the inner iterations (not while kernels are timed one by one
    // or traced: both need the individual launches on the caller's stream)
    static const bool dbg2 = std::getenv("DLMA_LOG") && std::getenv("DLMA_LOG")[0] == '2';
    const bool use_graph = o.graph_iters > 0 && !Profiler::get().on && !dbg2;
    IterGraph ig, igt;
    if (use_graph) check = o.graph_iters;
    // The first replay of a pass runs `check` iterations, the later ones `tail`: most
    // right-hand sides converge a few iterations after the first check, and every
    // iteration run after the last of them has converged still costs its launches
    // (about 1.1 ms at 24^3x48 with 192 right-hand sides, mostly blocks that find
    // nothing active).
    const int tail = std::min(check, 2);

    // After an odd-site reconstruction x_o += A_oo^-1 (r_o - D_oe e) the odd residual
    // b_o - A_oo x_o - D_oe x_e vanishes up to FP64 rounding.  Passes after one then
    // compute the residual on the even sites only, straight into the Schur source E
    // (with R_o = 0, T = A_oo^-1 R_o = 0 and E = R_e), and reconstruct without R_o.
    // When every right-hand side has converged on the even sites, the odd-site
    // residual of the same x completes the full norm that confirms it.
    bool odd_zero = false;
    // sites: 0 both parities, 1 even (odd partials 0), both for the right-hand sides of
    // the last pass (the others keep their norms); 2 odd sites of every right-hand
    // side, added to the norms held on the host
    // FP16 inner solves: the accumulation x_e += e of a pass is left to the even-site
    // residual that starts the next one (F_ACCX); acc_pending marks it as owed
    bool acc_pending = false;
    auto true_residual = [&](int sites) -> int {
        if (acc_pending && sites != 1) {  // not reached (the next residual is the even one); kept exact
            DLMA_HIP(launch_accum_to64<P>(t.dacc.template as<VecJob<P>>(), t.dacc64.template as<VecJob<P64>>(), t.nconv,
                                          t.bconv, s));
            acc_pending = false;
        }
        if (sites == 2) {
            for (auto& c : cs)
                DLMA_HIP(hipMemset2DAsync(c.part.as<double>(), 2 * sizeof(double) * c.hnsb, 0, sizeof(double) * c.hnsb,
                                          c.nrhs, s));
        }
        if (sites == 1) {
            for (auto& c : cs)  // the odd sites' partial norms are zero
                DLMA_HIP(hipMemset2DAsync(c.part.as<double>() + c.hnsb, 2 * sizeof(double) * c.hnsb, 0,
                                          sizeof(double) * c.hnsb, c.nrhs, s));
            DLMA_HIP(launch_hop<P64>(HopCfg{K2, F_HASB | F_NORM | (acc_pending ? F_ACCX : 0), t.nb64},
                                     t.dresidE.template as<HopJob<P64>>(), t.nresidE, t.bresidE, s));
            acc_pending = false;
        } else if (sites == 2) {
            DLMA_HIP(launch_hop<P64>(HopCfg{K2, F_HASB | F_NORM, t.nb64}, t.dresidO.template as<HopJob<P64>>(), t.nresidO,
                                     t.bresidO, s));
        } else {
            DLMA_HIP(launch_hop<P64>(HopCfg{K2, F_HASB | F_NORM, t.nb64}, t.dresid.template as<HopJob<P64>>(), t.nresid, t.bresid, s));
        }
        DLMA_HIP(launch_finish(t.dfinR.template as<FinJob>(), t.nfin, t.bfin, FIN_NORM, s));
        std::vector<std::vector<double>> got(cs.size());
        for (size_t i = 0; i < cs.size(); ++i) {
            got[i].resize(cs[i].nrhs);
            DLMA_HIP(hipMemcpyAsync(got[i].data(), cs[i].nrm, sizeof(double) * cs[i].nrhs, hipMemcpyDeviceToHost, s));
        }
        DLMA_HIP(hipStreamSynchronize(s));
        for (size_t i = 0; i < cs.size(); ++i)
            for (int r = 0; r < cs[i].nrhs; ++r) {
                Cfg& c = cs[i];
                if (sites == 2) {  // complete the norms that hold the even sites only
                    if (c.evenonly[r]) c.rnorm2[r] += got[i][r];
                    c.evenonly[r] = 0;
                } else if (c.hoact[r]) {
                    c.rnorm2[r] = got[i][r];
                    c.evenonly[r] = sites == 1;
                }
            }
        return DLMA_OK;
    };
    auto any_even_only = [&]() {
        for (auto& c : cs)
            for (char e : c.evenonly)
                if (e) return true;
        return false;
    };
    auto upload_oact = [&](bool all) -> int {
        for (auto& c : cs) {
            if (all) std::fill(c.hoact.begin(), c.hoact.end(), 1);
            DLMA_HIP(hipMemcpyAsync(c.oact, c.hoact.data(), sizeof(int) * c.nrhs, hipMemcpyHostToDevice, s));
        }
        return DLMA_OK;
    };
    DLMA_TRY(upload_oact(true));
    for (int pass = 0;; ++pass) {
        // true residual; from x = 0 it is b, and the first pass's jobs read B in place of R
        const bool from_b = pass == 0 && !o.use_x0;
        if (from_b) {
            for (auto& c : cs) c.rnorm2 = c.bnorm2;
        } else {
            DLMA_TRY(true_residual(odd_zero ? 1 : 0));
            if (odd_zero) {  // all converged on the even sites: add the odd sites of the same x
                bool all = true;
                for (auto& c : cs)
                    for (int r = 0; r < c.nrhs && all; ++r)
                        all = c.bnorm2[r] > 0 ? std::sqrt(c.rnorm2[r] / c.bnorm2[r]) <= o.tol : true;
                if (all) {
                    DLMA_TRY(true_residual(2));
                    bool still = true;
                    for (auto& c : cs)
                        for (int r = 0; r < c.nrhs && still; ++r)
                            still = c.bnorm2[r] > 0 ? std::sqrt(c.rnorm2[r] / c.bnorm2[r]) <= o.tol : true;
                    if (!still) {  // rounding left an odd residual: start over from the full one
                        odd_zero = false;
                        DLMA_TRY(upload_oact(true));
                        DLMA_TRY(true_residual(0));
                    }
                }
            }
        }
        int nleft = 0;
        int maxused = 0;
        auto evaluate = [&]() {
            nleft = 0;
            maxused = 0;
            for (auto& c : cs) {
                c.outer = pass;
                for (int r = 0; r < c.nrhs; ++r) {
                    double rr = c.rnorm2[r];
                    if (!std::isfinite(rr)) nan = true;
                    c.relres[r] = c.bnorm2[r] > 0 ? std::sqrt(rr / c.bnorm2[r]) : 0.0;
                    c.conv[r] = (c.relres[r] <= o.tol) ? 1 : 0;
                    if (!c.conv[r]) { ++nleft; maxused = std::max(maxused, c.used[r]); }
                    c.hact[r] = c.conv[r] ? 0 : 1;
                }
            }
        };
        evaluate();
        // stopped by a cap with even-site norms still held: the statistics report the
        // full residual of every right-hand side, so add the odd sites once
        if (!nan && nleft > 0 && (pass >= o.max_outer || maxused >= o.maxiter) && any_even_only()) {
            DLMA_TRY(true_residual(2));
            evaluate();
        }
        if (nan) return fail(DLMA_ENAN, "non-finite residual during the solve");
        if (dlog) {
            double mx = 0, mn = 1e300;
            for (auto& c : cs)
                for (double r : c.relres) { mx = std::max(mx, r); mn = std::min(mn, r); }
            std::fprintf(stderr, "[dlma] pass %d: %d rhs left, relres %.3e .. %.3e\n", pass, nleft, mn, mx);
        }
        if (nleft == 0 || pass >= o.max_outer || maxused >= o.maxiter) break;
        // right-hand sides iterated in this pass: the inner solver's flags and the mask
        // of the FP64 kernels (conversion, accumulation, reconstruction, next residual)
        for (auto& c : cs) {
            DLMA_HIP(hipMemcpyAsync(c.active, c.hact.data(), sizeof(int) * c.nrhs, hipMemcpyHostToDevice, s));
            c.hoact = c.hact;
        }
        DLMA_TRY(upload_oact(false));
        // Schur source E = R_e + 1/2 H_eo A_oo^-1 R_o and |E|^2; with R_o = 0 the
        // even-site residual already wrote E, and its norm is the residual's
        if (odd_zero) {
            for (auto& c : cs) DLMA_HIP(hipMemcpyAsync(c.enrm, c.nrm, sizeof(double) * c.nrhs, hipMemcpyDeviceToDevice, s));
        } else {
            DLMA_HIP(launch_clover_apply64((from_b ? t.dclov0 : t.dclov).template as<VecJob<P64>>(), t.nclov, t.bclov, s));
            DLMA_HIP(launch_hop<P64>(HopCfg{K2, F_NOA, t.nb64}, (from_b ? t.dprep0 : t.dprep).template as<HopJob<P64>>(),
                                     t.nprep, t.bprep, s));
            DLMA_HIP(launch_norm<P64>((from_b ? t.dvnE0 : t.dvnE).template as<VecJob<P64>>(), t.nconv, t.bvnE, s));
            DLMA_HIP(launch_finish(t.dfinE.template as<FinJob>(), t.nfin, t.bfin, FIN_NORM, s));
        }
        DLMA_HIP(launch_conv_from64<P>(t.dconv.template as<VecJob<P>>(), t.nconv, t.bconv,
                                       (from_b ? t.dconv640 : t.dconv64).template as<VecJob<P64>>(), s));
        for (auto& f : t.hfinI) { f.rel2 = rel * rel; f.maxit = std::max(1, o.maxiter - maxused); }
        for (auto& f : t.hfinAB) f.maxit = std::max(1, o.maxiter - maxused);
        DLMA_HIP(hipMemcpyAsync(t.dfinI.p, t.hfinI.data(), sizeof(FinJob) * t.hfinI.size(), hipMemcpyHostToDevice, s));
        DLMA_HIP(hipMemcpyAsync(t.dfinAB.p, t.hfinAB.data(), sizeof(FinJob) * t.hfinAB.size(), hipMemcpyHostToDevice, s));
        DLMA_HIP(launch_finish(t.dfinI.template as<FinJob>(), t.nfin, t.bfin, FIN_INIT, s));
        if (t.bicg) {  // rho = (rh, r) (p = r already), per-pass iteration caps
            for (auto& f : t.hbf) f.maxit = std::max(1, o.maxiter - maxused);
            DLMA_HIP(hipMemcpyAsync(t.dbf.p, t.hbf.data(), sizeof(BiFinJob) * t.hbf.size(), hipMemcpyHostToDevice, s));
            DLMA_HIP(launch_bivec<P>(t.dbv.template as<BiVecJob<P>>(), t.nbv, t.bbv, BV_RR, s));
            DLMA_HIP(launch_bifinish(t.dbf.template as<BiFinJob>(), t.nbv, t.bbf, BF_INIT, s));
        }
        const bool windowed = from_b && arcn > 0;
        if (reach_skip) {
            for (auto& c : cs) {
                if (from_b) {  // what the skipped sites and blocks leave untouched starts at zero:
                    // s (the s step), and with windowed stencils also y, v and t
                    for (Buf* f : {&c.bs, &c.nbs}) DLMA_HIP(hipMemsetAsync(f->p, 0, f->n, s));
                    if (windowed)
                        for (Buf* f : {&c.y, &c.ny, &c.w, &c.nw, &c.bt, &c.nbt}) DLMA_HIP(hipMemsetAsync(f->p, 0, f->n, s));
                } else if (pass == 1) {  // dense from here on: everything within reach
                    DLMA_HIP(hipMemsetAsync(c.tdist.p, 0, c.tdist.n, s));
                }
            }
        }
        std::vector<int> nact(ncfg);
        for (int i = 0; i < ncfg; ++i) nact[i] = (int)std::count(cs[i].hact.begin(), cs[i].hact.end(), 1);
        // First pass, one configuration: while K1 of p has not reached every timeslice,
        // iteration k launches its stencils over the sources' arc widened by their reach
        // (2 + 4k, 3 + 4k, 4 + 4k, 5 + 4k timeslices for K1 of p, K2 for v, K1 of s, K2 for
        // t); the vector steps skip site by site (in_reach).  These iterations run as
        // direct launches before the replays.
        if (windowed) {
            const int T = cs[0].g->geo.T;
            for (int k = 0;; ++k) {
                IterWin w;
                for (int i = 0; i < 4; ++i) {
                    const int rho = 2 + i + 4 * k, W = arcn + 2 * rho;
                    w.tw0[i] = W < T ? ((arc0 - rho) % T + T) % T : 0;
                    w.twn[i] = W < T ? W : 0;
                }
                if (w.twn[0] == 0) break;
                DLMA_TRY(bicg_iteration<P>(cs, t, nb, nact, s, &w));
            }
        }
        // inner CG
        if (use_graph && !ig.exec) DLMA_TRY(capture_iterations<P>(cs, t, nb, nact, check, ig));
        for (bool first = true;; first = false) {
            if (use_graph) {
                if (!first && !igt.exec) DLMA_TRY(capture_iterations<P>(cs, t, nb, nact, tail, igt));
                DLMA_HIP(hipGraphLaunch(first ? ig.exec : igt.exec, s));
            } else {
                for (int k = 0; k < (first ? check : tail); ++k) DLMA_TRY(inner_iteration<P>(cs, t, nb, nact, s));
            }
            int tot = 0;
            for (int i = 0; i < ncfg; ++i)
                DLMA_HIP(hipMemcpyAsync(cs[i].hact.data(), cs[i].active, sizeof(int) * cs[i].nrhs, hipMemcpyDeviceToHost, s));
            DLMA_HIP(hipStreamSynchronize(s));
            if (Profiler::get().on) Profiler::get().collect();
            for (int i = 0; i < ncfg; ++i) {
                nact[i] = (int)std::count(cs[i].hact.begin(), cs[i].hact.end(), 1);
                tot += nact[i];
            }
            if (dlog) {
                std::vector<double> rr(cs[0].nrhs), rr0(cs[0].nrhs), al(cs[0].nrhs);
                (void)hipMemcpy(rr.data(), cs[0].rr, sizeof(double) * cs[0].nrhs, hipMemcpyDeviceToHost);
                (void)hipMemcpy(rr0.data(), cs[0].rr0, sizeof(double) * cs[0].nrhs, hipMemcpyDeviceToHost);
                (void)hipMemcpy(al.data(), cs[0].alpha, sizeof(double) * cs[0].nrhs, hipMemcpyDeviceToHost);
                std::fprintf(stderr, "[dlma]   inner: %d active; rhs0 |r|^2 %.3e / %.3e alpha %.3e\n", tot, rr[0], rr0[0], al[0]);
            }
            if (tot == 0) break;
        }
        // reconstruction (FP16: the even sites' accumulation is fused into the next residual)
        if (P == P16) acc_pending = true;
        else DLMA_HIP(launch_accum_to64<P>(t.dacc.template as<VecJob<P>>(), t.dacc64.template as<VecJob<P64>>(), t.nconv, t.bconv, s));
        constexpr int in16 = P == P16 ? F_IN16 : 0;
        if (odd_zero)
            DLMA_HIP(launch_hop<P64>(HopCfg{K1, F_ACCUM | in16, t.nb64}, t.drecon.template as<HopJob<P64>>(), t.nrecon, t.brecon, s));
        else
            DLMA_HIP(launch_hop<P64>(HopCfg{K1, F_HASD | F_ACCUM | in16, t.nb64},
                                     (from_b ? t.drecon0 : t.drecon).template as<HopJob<P64>>(), t.nrecon, t.brecon, s));
        odd_zero = true;  // every right-hand side now has r_o = 0 up to rounding
        for (auto& c : cs) DLMA_HIP(hipMemcpyAsync(c.hiters.data(), c.iters, sizeof(int) * c.nrhs, hipMemcpyDeviceToHost, s));
        DLMA_HIP(hipStreamSynchronize(s));
        for (auto& c : cs)
            for (int r = 0; r < c.nrhs; ++r) c.used[r] += c.hiters[r];
    }
    for (auto& c : cs) DLMA_HIP(launch_eo_to_canon(c.X.as<double2>(), c.xcan, c.g->geo, c.nrhs, s, o.dagger));
    DLMA_HIP(hipStreamSynchronize(s));
    return DLMA_OK;
}

// Autotuner of the stencil launch shape: right-hand sides per thread (nb; fixed
// when the caller gives one) and right-hand-side groups per super-group (sg, the
// block order of hop_kernel); for FP16 fields also whether the stencils stage their
// LDS window (tried for the best nb and sg).  Each candidate times the Schur pair
// K1 + K2 on the caller's buffers (vp filled with random numbers): one warm-up and
// five timed repetitions, median.  Results are cached per lattice, precision,
// right-hand sides and fixed nb for the life of the process.
template <int P> int tune_hop(Gauge* g, int nrhs, int fixed_nb, SF<P> vp, SF<P> vy, SF<P> vw, Tune& out, hipStream_t s) {
    const int key = P * 16 + fixed_nb;
    if (int v = tuned_lookup(g->dims, key, nrhs)) {
        out.nb = v & 255;
        out.sg = (v >> 8) & 255;
        out.win = v >> 16;
        return DLMA_OK;
    }
    DLMA_HIP(launch_fill_random<P>(vp, g->Vh, nrhs, 7u, s));
    struct Ev {  // released on every return path
        hipEvent_t e = nullptr;
        ~Ev() { if (e) (void)hipEventDestroy(e); }
    } ev0, ev1;
    DLMA_HIP(hipEventCreate(&ev0.e));
    DLMA_HIP(hipEventCreate(&ev1.e));
    hipEvent_t e0 = ev0.e, e1 = ev1.e;
    static const bool tlog = std::getenv("DLMA_LOG") != nullptr;
    auto time_cfg = [&](const Tune& c, float& med) -> int {
        std::vector<HopJob<P>> k1v, k2v;
        HopJob<P> j1 = hop_job<P>(g, 1, nrhs, c.nb, c.win != 0);
        j1.U = (const typename PT<P>::S*)gauge_links(g, P);
        j1.C = (const typename PT<P>::S*)gauge_clover_oo_inv(g, P);
        j1.ch = -0.5;
        j1.in = vp;
        j1.out = vy;
        j1.sg = c.sg;
        HopJob<P> j2 = hop_job<P>(g, 0, nrhs, c.nb, c.win != 0);
        j2.U = j1.U;
        j2.C = (const typename PT<P>::S*)gauge_clover_ee(g, P);
        j2.ca = 1.0;
        j2.ch = 0.5;
        j2.x = vp;
        j2.in = vy;
        j2.out = vw;
        j2.sg = c.sg;
        k1v.push_back(j1);
        k2v.push_back(j2);
        int b1 = assign_blocks(k1v), b2 = assign_blocks(k2v);
        Buf d1, d2;
        DLMA_TRY(upload(d1, k1v, s));
        DLMA_TRY(upload(d2, k2v, s));
        std::vector<float> ts;
        for (int rep = 0; rep < 6; ++rep) {
            DLMA_HIP(hipEventRecord(e0, s));
            DLMA_HIP(launch_hop<P>(HopCfg{K1, 0, c.nb, j1.wn}, d1.as<HopJob<P>>(), 1, b1, s));
            DLMA_HIP(launch_hop<P>(HopCfg{K2, 0, c.nb, j2.wn}, d2.as<HopJob<P>>(), 1, b2, s));
            DLMA_HIP(hipEventRecord(e1, s));
            DLMA_HIP(hipEventSynchronize(e1));
            float ms = 0;
            DLMA_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) ts.push_back(ms);
        }
        DLMA_HIP(hipStreamSynchronize(s));
        std::sort(ts.begin(), ts.end());
        med = ts[ts.size() / 2];
        if (tlog)
            std::fprintf(stderr, "[dlma] tune prec %d nrhs %d Vh %d: nb %d sg %d window %d -> %.3f ms (K1+K2)\n", P, nrhs, g->Vh,
                         c.nb, c.sg, j1.wn > 0 ? 1 : 0, med);
        return DLMA_OK;
    };
    Tune best{1, 0, 1};
    float bt = 1e30f;
    const int nbs[4] = {1, 2, 3, 4};
    const int sgs[7] = {1, 2, 4, 8, 16, 32, 0};
    for (int nb : nbs) {
        if (fixed_nb && nb != fixed_nb) continue;
        if (!fixed_nb && nb > 1 && nrhs < nb) continue;
        const int G = ceil_div(nrhs, nb);
        for (int sg : sgs) {
            if (sg >= G) continue;  // same order as sg = 0 (all groups)
            float med = 0;
            DLMA_TRY(time_cfg(Tune{nb, sg, 1}, med));
            if (med < bt) {
                bt = med;
                best = Tune{nb, sg, 1};
            }
        }
    }
    if (P == P16 && hop_job<P>(g, 0, nrhs, best.nb).wn > 0) {
        float med = 0;
        DLMA_TRY(time_cfg(Tune{best.nb, best.sg, 0}, med));
        if (med < bt) best.win = 0;
    }
    tuned_store(g->dims, key, nrhs, best.nb | (best.sg << 8) | (best.win << 16));
    out = best;
    return DLMA_OK;
}

}  // namespace

extern "C" int dlma_solve(const dlma_gauge_t* gs, int ngauge, const dlma_rhs_set* sets, const dlma_solve_opts* opts,
                          dlma_solve_stat* stats, void* stream) {
    if (!gs || !sets || ngauge < 1 || ngauge > MAXG) return fail(DLMA_EINVAL, "need 1..16 gauge handles and rhs sets");
    dlma_solve_opts o;
    if (opts) o = *opts;
    else dlma_solve_opts_default(&o);
    if (!(o.tol > 0.0) || !std::isfinite(o.tol)) return fail(DLMA_EINVAL, "tol must be positive");
    if (o.maxiter < 1 || o.max_outer < 0) return fail(DLMA_EINVAL, "maxiter must be >= 1 and max_outer >= 0");
    if (o.prec < 0 || o.prec > 3) return fail(DLMA_EINVAL, "prec must be one of DLMA_PREC_*");
    if (o.inner_tol < 0 || o.inner_tol >= 1) return fail(DLMA_EINVAL, "inner_tol must be in [0, 1)");
    if (o.check_every < 0 || o.graph_iters < 0) return fail(DLMA_EINVAL, "check_every and graph_iters must be >= 0");
    if (o.dagger != 0 && o.dagger != 1) return fail(DLMA_EINVAL, "dagger must be 0 or 1");
    if (o.lds_window < -1 || o.lds_window > 1) return fail(DLMA_EINVAL, "lds_window must be -1, 0 or 1");
    if (o.inner_solver < 0 || o.inner_solver > 1) return fail(DLMA_EINVAL, "inner_solver must be 0 (CGNE) or 1 (BiCGStab)");
    std::vector<Cfg> cs;
    cs.reserve(ngauge);
    int total = 0;
    for (int i = 0; i < ngauge; ++i) {
        if (!gs[i]) return fail(DLMA_EINVAL, "NULL gauge handle");
        if (sets[i].nrhs < 0) return fail(DLMA_EINVAL, "nrhs < 0");
        if (sets[i].nrhs == 0) continue;
        if (!sets[i].b || !sets[i].x) return fail(DLMA_EINVAL, "NULL b or x");
        cs.emplace_back();
        Cfg& c = cs.back();
        c.g = (Gauge*)gs[i];
        c.nrhs = sets[i].nrhs;
        c.gidx = i;
        c.bcan = (const double2*)sets[i].b;
        c.xcan = (double2*)sets[i].x;
        total += c.nrhs;
    }
    if (cs.empty()) return DLMA_OK;
    // gauge handles may repeat only with distinct outputs; outputs must not alias inputs
    hipStream_t s = S(stream);
    int rc;
    switch (o.prec) {
    case DLMA_PREC_FP64: rc = solve_impl<P64>(cs, o, s); break;
    case DLMA_PREC_MIX_FP32: rc = solve_impl<P32>(cs, o, s); break;
    case DLMA_PREC_MIX_FP16: rc = solve_impl<P16>(cs, o, s); break;
    default: rc = solve_impl<PB16>(cs, o, s); break;
    }
    if (rc != DLMA_OK && rc != DLMA_ENOTCONV) {
        (void)hipStreamSynchronize(s);
        return rc;
    }
    bool allconv = true;
    if (stats) {
        // stats in the order of the sets (sets with nrhs == 0 contribute nothing)
        int k = 0;
        for (auto& c : cs)
            for (int r = 0; r < c.nrhs; ++r, ++k) {
                stats[k].outer = c.outer;
                stats[k].inner_iters = c.used[r];
                stats[k].relres = c.relres[r];
                stats[k].converged = c.conv[r];
            }
    }
    for (auto& c : cs)
        for (int r = 0; r < c.nrhs; ++r) allconv = allconv && c.conv[r];
    (void)total;
    if (!allconv) return fail(DLMA_ENOTCONV, "not every right-hand side reached the tolerance");
    return DLMA_OK;
}

// ---------------------------------------------------------------- Schur benchmark

namespace {
template <int P>
int bench_impl(Gauge* g, int nrhs, int nb, int napply, double* ms_out, double* bytes_out, hipStream_t s) {
    DLMA_TRY(gauge_prepare(g, P, s));
    int Vh = g->Vh;
    size_t halfP = pair_bytes(P) * (size_t)nrhs * 12 * Vh;
    Buf a, y, w, na, ny, nw;
    DLMA_TRY(a.allocate(halfP));
    DLMA_TRY(y.allocate(halfP));
    DLMA_TRY(w.allocate(halfP));
    if (P == P16) {
        DLMA_TRY(na.allocate(sizeof(float) * nrhs * Vh));
        DLMA_TRY(ny.allocate(sizeof(float) * nrhs * Vh));
        DLMA_TRY(nw.allocate(sizeof(float) * nrhs * Vh));
    }
    SF<P> va = half_view<P>(a.p, nrm_of<P>(na), Vh), vy = half_view<P>(y.p, nrm_of<P>(ny), Vh),
          vw = half_view<P>(w.p, nrm_of<P>(nw), Vh);
    DLMA_HIP(launch_fill_random<P>(va, Vh, nrhs, 11u, s));
    Tune tn{nb ? nb : 1, 0, 1};
    DLMA_TRY(tune_hop<P>(g, nrhs, nb, va, vy, vw, tn, s));
    nb = tn.nb;
    DLMA_HIP(launch_fill_random<P>(va, Vh, nrhs, 11u, s));
    // alternate Dhat and Dhat^dag: a -> w -> a
    std::vector<HopJob<P>> j1f, j2f, j1b, j2b;
    HopJob<P> j1 = hop_job<P>(g, 1, nrhs, nb, tn.win != 0);
    j1.U = (const typename PT<P>::S*)gauge_links(g, P);
    j1.C = (const typename PT<P>::S*)gauge_clover_oo_inv(g, P);
    j1.ch = -0.5;
    j1.sg = tn.sg;
    HopJob<P> j2 = hop_job<P>(g, 0, nrhs, nb, tn.win != 0);
    j2.sg = tn.sg;
    j2.U = j1.U;
    j2.C = (const typename PT<P>::S*)gauge_clover_ee(g, P);
    j2.ca = 1.0;
    j2.ch = 0.5;
    HopJob<P> t1 = j1; t1.in = va; t1.out = vy; j1f.push_back(t1);
    HopJob<P> t2 = j2; t2.x = va; t2.in = vy; t2.out = vw; j2f.push_back(t2);
    HopJob<P> t3 = j1; t3.in = vw; t3.out = vy; j1b.push_back(t3);
    HopJob<P> t4 = j2; t4.x = vw; t4.in = vy; t4.out = va; j2b.push_back(t4);
    int b1 = assign_blocks(j1f); assign_blocks(j1b);
    int b2 = assign_blocks(j2f); assign_blocks(j2b);
    Buf d1f, d2f, d1b, d2b;
    DLMA_TRY(upload(d1f, j1f, s)); DLMA_TRY(upload(d2f, j2f, s));
    DLMA_TRY(upload(d1b, j1b, s)); DLMA_TRY(upload(d2b, j2b, s));
    double by1 = hop_bytes(P, K1, 0, Vh, nrhs), by2 = hop_bytes(P, K2, 0, Vh, nrhs);
    auto run = [&](int k) -> int {
        bool fwd = (k & 1) == 0;
        DLMA_TRY(hop_launch<P>(HopCfg{K1, fwd ? 0 : F_G5IN, nb, j1.wn}, (fwd ? d1f : d1b).p, 1, b1, fwd ? KC_K1 : KC_K1DAG, by1, s));
        DLMA_TRY(hop_launch<P>(HopCfg{K2, fwd ? 0 : F_G5OUT, nb, j2.wn}, (fwd ? d2f : d2b).p, 1, b2, KC_K2, by2, s));
        return DLMA_OK;
    };
    DLMA_TRY(run(0));
    DLMA_TRY(run(1));
    DLMA_HIP(hipStreamSynchronize(s));
    if (Profiler::get().on) Profiler::get().collect();
    struct Ev {  // released on every return path
        hipEvent_t e = nullptr;
        ~Ev() { if (e) (void)hipEventDestroy(e); }
    } ev0, ev1;
    DLMA_HIP(hipEventCreate(&ev0.e));
    DLMA_HIP(hipEventCreate(&ev1.e));
    hipEvent_t e0 = ev0.e, e1 = ev1.e;
    DLMA_HIP(hipEventRecord(e0, s));
    for (int k = 0; k < napply; ++k) DLMA_TRY(run(k));
    DLMA_HIP(hipEventRecord(e1, s));
    DLMA_HIP(hipEventSynchronize(e1));
    float ms = 0;
    DLMA_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    DLMA_HIP(hipStreamSynchronize(s));
    if (Profiler::get().on) Profiler::get().collect();
    if (ms_out) *ms_out = ms / napply;
    if (bytes_out) *bytes_out = by1 + by2;
    return DLMA_OK;
}
}  // namespace

// ---------------------------------------------------------------- Schur operator

namespace {
// out_e = Dhat in_e (or Dhat^dag in_e) with the inner stencils of precision P: the
// even sites of `in` rounded to P at scale 1 by the solver's conversion kernel, the
// solver's K1 and K2 launches, the result widened to FP64; odd sites of out are 0.
template <int P>
int schur_impl(Gauge* g, const void* in, void* out, int nrhs, int dagger, int nb, int sg, int win, hipStream_t s) {
    DLMA_TRY(gauge_prepare(g, P, s));
    const int Vh = g->Vh;
    const size_t full64 = sizeof(double2) * (size_t)nrhs * 24 * Vh;
    const size_t halfP = pair_bytes(P) * (size_t)nrhs * 12 * Vh;
    const int vnsb = ceil_div(Vh, VEC_BS);
    Buf a64, b64, a, y, w, na, ny, nw, ones, part;
    DLMA_TRY(a64.allocate(full64));
    DLMA_TRY(b64.allocate(full64));
    DLMA_TRY(a.allocate(halfP));
    DLMA_TRY(y.allocate(halfP));
    DLMA_TRY(w.allocate(halfP));
    if (P == P16) {
        DLMA_TRY(na.allocate(sizeof(float) * nrhs * Vh));
        DLMA_TRY(ny.allocate(sizeof(float) * nrhs * Vh));
        DLMA_TRY(nw.allocate(sizeof(float) * nrhs * Vh));
    }
    DLMA_TRY(part.allocate(sizeof(double) * (size_t)nrhs * vnsb));
    DLMA_TRY(upload(ones, std::vector<double>((size_t)nrhs, 1.0), s));
    SF<P> va = half_view<P>(a.p, nrm_of<P>(na), Vh), vy = half_view<P>(y.p, nrm_of<P>(ny), Vh),
          vw = half_view<P>(w.p, nrm_of<P>(nw), Vh);
    if (nb == 0) {  // the solver's launch shape (the tuner overwrites va)
        Tune tn{1, 0, 1};
        DLMA_TRY(tune_hop<P>(g, nrhs, 0, va, vy, vw, tn, s));
        nb = tn.nb;
        sg = tn.sg;
        win = tn.win;
    }
    DLMA_HIP(launch_canon_to_eo((const double2*)in, a64.as<double2>(), g->geo, nrhs, s));
    VecJob<P> cv = {};
    cv.Vh = Vh; cv.nrhs = nrhs; cv.nsb = vnsb;
    cv.a = va; cv.b = vw; cv.c = vy;  // b and c are scratch here
    cv.s = ones.as<double>();
    cv.part = part.as<double>(); cv.pstride = vnsb;
    VecJob<P64> cv64 = {};
    cv64.Vh = Vh; cv64.nrhs = nrhs; cv64.nsb = vnsb;
    cv64.a = full_view(a64.p, Vh, 0);
    VecJob<P> ac = cv;
    ac.a = vw;
    VecJob<P64> ac64 = cv64;
    ac64.a = full_view(b64.p, Vh, 0);
    ac64.b = full_view(a64.p, Vh, 0);  // accumulator of the kernel, scratch here
    std::vector<VecJob<P>> cvv{cv}, acv{ac};
    std::vector<VecJob<P64>> cv64v{cv64}, ac64v{ac64};
    const int bconv = assign_vec_blocks(cvv);
    assign_vec_blocks(acv); assign_vec_blocks(cv64v); assign_vec_blocks(ac64v);
    HopJob<P> j1 = hop_job<P>(g, 1, nrhs, nb, win != 0);
    j1.U = (const typename PT<P>::S*)gauge_links(g, P);
    j1.C = (const typename PT<P>::S*)gauge_clover_oo_inv(g, P);
    j1.ch = -0.5;
    j1.sg = sg;
    j1.in = va;
    j1.out = vy;
    HopJob<P> j2 = hop_job<P>(g, 0, nrhs, nb, win != 0);
    j2.U = j1.U;
    j2.C = (const typename PT<P>::S*)gauge_clover_ee(g, P);
    j2.ca = 1.0;
    j2.ch = 0.5;
    j2.sg = sg;
    j2.x = va;
    j2.in = vy;
    j2.out = vw;
    std::vector<HopJob<P>> k1v{j1}, k2v{j2};
    const int b1 = assign_blocks(k1v), b2 = assign_blocks(k2v);
    Buf dcv, dac, dcv64, dac64, d1, d2;
    DLMA_TRY(upload(dcv, cvv, s)); DLMA_TRY(upload(dac, acv, s));
    DLMA_TRY(upload(dcv64, cv64v, s)); DLMA_TRY(upload(dac64, ac64v, s));
    DLMA_TRY(upload(d1, k1v, s)); DLMA_TRY(upload(d2, k2v, s));
    DLMA_HIP(launch_conv_from64<P>(dcv.as<VecJob<P>>(), 1, bconv, dcv64.as<VecJob<P64>>(), s));
    DLMA_HIP(launch_hop<P>(HopCfg{K1, dagger ? F_G5IN : 0, nb, j1.wn}, d1.as<HopJob<P>>(), 1, b1, s));
    DLMA_HIP(launch_hop<P>(HopCfg{K2, dagger ? F_G5OUT : 0, nb, j2.wn}, d2.as<HopJob<P>>(), 1, b2, s));
    DLMA_HIP(hipMemsetAsync(b64.p, 0, full64, s));
    DLMA_HIP(launch_accum_to64<P>(dac.as<VecJob<P>>(), dac64.as<VecJob<P64>>(), 1, bconv, s));
    DLMA_HIP(launch_eo_to_canon(b64.as<double2>(), (double2*)out, g->geo, nrhs, s));
    DLMA_HIP(hipStreamSynchronize(s));
    return DLMA_OK;
}
}  // namespace

extern "C" int dlma_apply_schur(dlma_gauge_t h, const void* in, void* out, int nrhs, int dagger, int prec, int rhs_block,
                                int super_group, int lds_window, void* stream) {
    Gauge* g = (Gauge*)h;
    if (!g) return fail(DLMA_EINVAL, "NULL handle");
    if (nrhs < 0) return fail(DLMA_EINVAL, "nrhs < 0");
    if (nrhs == 0) return DLMA_OK;
    if (!in || !out) return fail(DLMA_EINVAL, "NULL field pointer");
    const size_t bytes = sizeof(double2) * (size_t)nrhs * 24 * g->Vh;
    const char *pi = (const char*)in, *po = (const char*)out;
    if (pi < po + bytes && po < pi + bytes) return fail(DLMA_EINVAL, "in and out must not overlap");
    if (dagger != 0 && dagger != 1) return fail(DLMA_EINVAL, "dagger must be 0 or 1");
    if (rhs_block < 0 || rhs_block > 4) return fail(DLMA_EINVAL, "rhs_block must be 0 .. 4");
    if (super_group < 0) return fail(DLMA_EINVAL, "super_group must be >= 0");
    if (lds_window != 0 && lds_window != 1) return fail(DLMA_EINVAL, "lds_window must be 0 or 1");
    hipStream_t s = S(stream);
    switch (prec) {
    case DLMA_PREC_FP64: return schur_impl<P64>(g, in, out, nrhs, dagger, rhs_block, super_group, lds_window, s);
    case DLMA_PREC_MIX_FP32: return schur_impl<P32>(g, in, out, nrhs, dagger, rhs_block, super_group, lds_window, s);
    case DLMA_PREC_MIX_FP16: return schur_impl<P16>(g, in, out, nrhs, dagger, rhs_block, super_group, lds_window, s);
    case DLMA_PREC_MIX_BF16: return schur_impl<PB16>(g, in, out, nrhs, dagger, rhs_block, super_group, lds_window, s);
    default: return fail(DLMA_EINVAL, "prec must be one of DLMA_PREC_*");
    }
}

extern "C" int dlma_bench_schur(dlma_gauge_t h, int prec, int nrhs, int rhs_block, int napply, double* ms_out,
                                double* bytes_out, void* stream) {
    Gauge* g = (Gauge*)h;
    if (!g) return fail(DLMA_EINVAL, "NULL handle");
    if (nrhs < 1 || napply < 1) return fail(DLMA_EINVAL, "nrhs and napply must be >= 1");
    if (rhs_block < 0 || rhs_block > 4) return fail(DLMA_EINVAL, "rhs_block must be 0 .. 4");
    hipStream_t s = S(stream);
    switch (prec) {
    case DLMA_PREC_FP64: return bench_impl<P64>(g, nrhs, rhs_block, napply, ms_out, bytes_out, s);
    case DLMA_PREC_MIX_FP32: return bench_impl<P32>(g, nrhs, rhs_block, napply, ms_out, bytes_out, s);
    case DLMA_PREC_MIX_FP16: return bench_impl<P16>(g, nrhs, rhs_block, napply, ms_out, bytes_out, s);
    case DLMA_PREC_MIX_BF16: return bench_impl<PB16>(g, nrhs, rhs_block, napply, ms_out, bytes_out, s);
    default: return fail(DLMA_EINVAL, "prec must be one of DLMA_PREC_*");
    }
}

extern "C" int dlma_bench_copy(long bytes, int reps, double* ms_out, void* stream) {
    if (bytes < 16 || bytes % 16 != 0 || reps < 1 || !ms_out)
        return fail(DLMA_EINVAL, "bytes must be a positive multiple of 16, reps >= 1, ms_out not NULL");
    hipStream_t s = S(stream);
    Buf a, b;
    DLMA_TRY(a.allocate((size_t)bytes));
    DLMA_TRY(b.allocate((size_t)bytes));
    DLMA_HIP(hipMemsetAsync(a.p, 0, (size_t)bytes, s));
    DLMA_HIP(launch_stream_copy(a.p, b.p, bytes / 16, s));  // warm-up
    hipEvent_t e0, e1;
    DLMA_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(DLMA_EHIP, "hipEventCreate failed");
    }
    hipError_t e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_stream_copy(a.p, b.p, bytes / 16, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(DLMA_EHIP, std::string("stream copy: ") + hipGetErrorString(e));
    *ms_out = ms / reps;
    return DLMA_OK;
}
