// Site-local steps and scalar finishers of BiCGStab on the even-odd reduced operator
// Dhat (the alternative inner solver of dlma_solve).  One iteration is
//   v = Dhat p;            alpha = rho / (rh, v)
//   s = r - alpha v;       t = Dhat s;       omega = (t, s) / (t, t)
//   x += alpha p + omega s;  r = s - omega t;  rho' = (rh, r);  beta = (rho'/rho)(alpha/omega)
//   p = r + beta (p - omega v)
// with (a, b) = sum conj(a_i) b_i over the even sites.  The operator applications
// are the solver's stencil kernels; everything here is a streaming pass over fields
// of the storage precision, in FP64 arithmetic, with deterministic two-stage sums.
// The shadow residual rh is a fixed seeded random field rather than the initial
// residual: a distillation source lives on one timeslice and one spin, and with
// rh = r_0 the scalar (rh, r) loses almost all of the spreading residual, which
// leaves the FP16 recursion to drift from the true residual.  Every right-hand
// side of a configuration reads the same field (its views have RHS stride 0), so
// the x/r update and K2 with (rh, v) read it once per site rather than per RHS.
#include "kernels.h"

namespace dlma {

namespace {

struct Cd { double r, i; };
HD Cd cmulc(Cd a, Cd b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
HD Cd cdivc(Cd a, Cd b) {
    const double d = b.r * b.r + b.i * b.i;
    return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}
HD Cd ld2(const double2* p, int r) { const double2 v = p[r]; return {v.x, v.y}; }
HD bool finite2(Cd a) { return isfinite(a.r) && isfinite(a.i); }

// block sum of v written by thread 0 at part[idx]; every thread of the block calls it
__device__ __forceinline__ void bi_partial(double v, double* part, long idx) {
    __shared__ double lds[VEC_BS / 64];
    const double s = block_sum<VEC_BS>(v, lds);
    if (threadIdx.x == 0) part[idx] = s;
}

}  // namespace

// FP16 fields: the steps of one iteration in FP32 arithmetic on the raw words (128-bit
// loads and stores of the grouped layout, scales folded into the arithmetic).  FP32
// carries the 11-bit storage values and the FP64 scalars with margin; the partial
// sums are added in FP64.  Returns the NQ partial-sum contributions of the site.
HD void bv16_cplx(const uint32_t w[12], float n, float v[24]) {
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        v[2 * c] = lo16(w[c]) * n;
        v[2 * c + 1] = hi16(w[c]) * n;
    }
}

template <int MODE> HD void bivec16(const BiVecJob<P16>& J, int r, uint32_t site, double& q0, double& q1, double& q2) {
    const uint32_t Vh = (uint32_t)J.Vh, G16 = 16u * Vh, s16 = 16u * site, lo = 4u * site;
    uint32_t wa[12], wb[12], wc[12];
    float a[24], b[24], c[24];
    if (MODE == BV_S) {  // s = r - alpha v
        const F16Field R = f16_field(J.r, J.Vh, r), V = f16_field(J.v, J.Vh, r), S = f16_field(J.s, J.Vh, r);
        const float ar = (float)J.alpha[r].x, ai = (float)J.alpha[r].y;
        load_words<CP_NT>(R, s16, G16, wa);
        load_words<CP_NT>(V, s16, G16, wb);
        const float nr = wldf<CP_NT>(R.n, lo, 0), nv = wldf<CP_NT>(V.n, lo, 0);
        bv16_cplx(wa, nr, a);
        bv16_cplx(wb, nv, b);
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            c[2 * i] = a[2 * i] - (ar * b[2 * i] - ai * b[2 * i + 1]);
            c[2 * i + 1] = a[2 * i + 1] - (ar * b[2 * i + 1] + ai * b[2 * i]);
        }
        (void)store16(S, G16, site, c);
    } else if (MODE == BV_XR) {  // x += alpha p + omega s; r = s - omega t; |r|^2, (rh, r)
        const F16Field X = f16_field(J.x, J.Vh, r), Pp = f16_field(J.p, J.Vh, r), S = f16_field(J.s, J.Vh, r);
        const F16Field T = f16_field(J.t, J.Vh, r), R = f16_field(J.r, J.Vh, r), RH = f16_field(J.rh, J.Vh, r);
        const float alr = (float)J.alpha[r].x, ali = (float)J.alpha[r].y;
        const float omr = (float)J.omega[r].x, omi = (float)J.omega[r].y;
        // every load first (the stores to x and r could alias them as far as the
        // compiler can tell, which would otherwise hold the later loads behind them)
        uint32_t wt[12], wh[12];
        load_words<CP_NT>(X, s16, G16, wa);
        load_words<CP_NT>(Pp, s16, G16, wb);
        load_words<CP_NT>(S, s16, G16, wc);
        load_words<CP_NT>(T, s16, G16, wt);
        load_words(RH, s16, G16, wh);  // cached: every RHS reads this one field
        const float nx = wldf<CP_NT>(X.n, lo, 0), np = wldf<CP_NT>(Pp.n, lo, 0), ns = wldf<CP_NT>(S.n, lo, 0);
        const float nt = wldf<CP_NT>(T.n, lo, 0), nh = wldf(RH.n, lo, 0);
        bv16_cplx(wa, nx, a);
        bv16_cplx(wb, np, b);
        bv16_cplx(wc, ns, c);
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            const float pr = b[2 * i], pi = b[2 * i + 1], sr = c[2 * i], si = c[2 * i + 1];
            a[2 * i] += alr * pr - ali * pi + omr * sr - omi * si;
            a[2 * i + 1] += alr * pi + ali * pr + omr * si + omi * sr;
        }
        bv16_cplx(wt, nt, b);
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            const float tr = b[2 * i], ti = b[2 * i + 1];
            c[2 * i] -= omr * tr - omi * ti;
            c[2 * i + 1] -= omr * ti + omi * tr;
        }
        (void)store16(X, G16, site, a);
        // |r|^2 and (rh, r) of the new residual before its storage rounding
        q0 = (double)store16(R, G16, site, c);
        for (int i = 0; i < 12; ++i) wa[i] = wh[i];
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            const float hr = lo16(wa[i]), hi = hi16(wa[i]), rr = c[2 * i], ri = c[2 * i + 1];
            re = __builtin_fmaf(hr, rr, __builtin_fmaf(hi, ri, re));
            im = __builtin_fmaf(hr, ri, __builtin_fmaf(-hi, rr, im));
        }
        q1 = (double)re * nh;
        q2 = (double)im * nh;
    } else if (MODE == BV_SH) {  // s = r - alpha v, and (rh, s) of the stored s
        const F16Field R = f16_field(J.r, J.Vh, r), V = f16_field(J.v, J.Vh, r), S = f16_field(J.s, J.Vh, r);
        const F16Field RH = f16_field(J.rh, J.Vh, r);
        const float ar = (float)J.alpha[r].x, ai = (float)J.alpha[r].y;
        uint32_t wh[12];
        load_words<CP_NT>(R, s16, G16, wa);
        load_words<CP_NT>(V, s16, G16, wb);
        load_words(RH, s16, G16, wh);  // cached: every RHS reads this one field
        const float nr = wldf<CP_NT>(R.n, lo, 0), nv = wldf<CP_NT>(V.n, lo, 0), nh = wldf(RH.n, lo, 0);
        bv16_cplx(wa, nr, a);
        bv16_cplx(wb, nv, b);
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            c[2 * i] = a[2 * i] - (ar * b[2 * i] - ai * b[2 * i + 1]);
            c[2 * i + 1] = a[2 * i + 1] - (ar * b[2 * i + 1] + ai * b[2 * i]);
        }
        float ms;
        (void)store16w(S, G16, site, c, wc, ms);
        float re, im;
        dot16(wh, wc, re, im);
        q0 = (double)re * ((double)nh * ms);
        q1 = (double)im * ((double)nh * ms);
    } else if (MODE == BV_XRP) {  // x += alpha p + omega s; r = s - omega t; p = r + beta (p - omega v); |r|^2
        const F16Field X = f16_field(J.x, J.Vh, r), Pp = f16_field(J.p, J.Vh, r), S = f16_field(J.s, J.Vh, r);
        const F16Field T = f16_field(J.t, J.Vh, r), R = f16_field(J.r, J.Vh, r), V = f16_field(J.v, J.Vh, r);
        const float alr = (float)J.alpha[r].x, ali = (float)J.alpha[r].y;
        const float omr = (float)J.omega[r].x, omi = (float)J.omega[r].y;
        const float ber = (float)J.beta[r].x, bei = (float)J.beta[r].y;
        // every load first (the stores could alias them as far as the compiler can tell)
        uint32_t wt[12], wv[12];
        load_words<CP_NT>(X, s16, G16, wa);
        load_words<CP_NT>(Pp, s16, G16, wb);
        load_words<CP_NT>(S, s16, G16, wc);
        load_words<CP_NT>(T, s16, G16, wt);
        load_words<CP_NT>(V, s16, G16, wv);
        const float nx = wldf<CP_NT>(X.n, lo, 0), np = wldf<CP_NT>(Pp.n, lo, 0), ns = wldf<CP_NT>(S.n, lo, 0);
        const float nt = wldf<CP_NT>(T.n, lo, 0), nv = wldf<CP_NT>(V.n, lo, 0);
        bv16_cplx(wa, nx, a);
        bv16_cplx(wb, np, b);
        bv16_cplx(wc, ns, c);
#pragma unroll
        for (int i = 0; i < 12; ++i) {  // x += alpha p + omega s
            const float pr = b[2 * i], pi = b[2 * i + 1], sr = c[2 * i], si = c[2 * i + 1];
            a[2 * i] += alr * pr - ali * pi + omr * sr - omi * si;
            a[2 * i + 1] += alr * pi + ali * pr + omr * si + omi * sr;
        }
        (void)store16(X, G16, site, a);
        bv16_cplx(wt, nt, a);
#pragma unroll
        for (int i = 0; i < 12; ++i) {  // r = s - omega t
            const float tr = a[2 * i], ti = a[2 * i + 1];
            c[2 * i] -= omr * tr - omi * ti;
            c[2 * i + 1] -= omr * ti + omi * tr;
        }
        q0 = (double)store16(R, G16, site, c);
        bv16_cplx(wv, nv, a);
#pragma unroll
        for (int i = 0; i < 12; ++i) {  // p = r + beta (p - omega v)
            const float dr = b[2 * i] - (omr * a[2 * i] - omi * a[2 * i + 1]);
            const float di = b[2 * i + 1] - (omr * a[2 * i + 1] + omi * a[2 * i]);
            b[2 * i] = c[2 * i] + ber * dr - bei * di;
            b[2 * i + 1] = c[2 * i + 1] + ber * di + bei * dr;
        }
        (void)store16(Pp, G16, site, b);
    } else {  // BV_P: p = r + beta (p - omega v)
        const F16Field R = f16_field(J.r, J.Vh, r), Pp = f16_field(J.p, J.Vh, r), V = f16_field(J.v, J.Vh, r);
        const float ber = (float)J.beta[r].x, bei = (float)J.beta[r].y;
        const float omr = (float)J.omega[r].x, omi = (float)J.omega[r].y;
        load_words<CP_NT>(R, s16, G16, wa);
        load_words<CP_NT>(Pp, s16, G16, wb);
        load_words<CP_NT>(V, s16, G16, wc);
        const float nr = wldf<CP_NT>(R.n, lo, 0), np = wldf<CP_NT>(Pp.n, lo, 0), nv = wldf<CP_NT>(V.n, lo, 0);
        bv16_cplx(wa, nr, a);
        bv16_cplx(wb, np, b);
        bv16_cplx(wc, nv, c);
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            const float dr = b[2 * i] - (omr * c[2 * i] - omi * c[2 * i + 1]);
            const float di = b[2 * i + 1] - (omr * c[2 * i + 1] + omi * c[2 * i]);
            b[2 * i] = a[2 * i] + ber * dr - bei * di;
            b[2 * i + 1] = a[2 * i + 1] + ber * di + bei * dr;
        }
        (void)store16(Pp, G16, site, b);
    }
}

template <int P, int MODE> __global__ void __launch_bounds__(VEC_BS) k_bivec(const BiVecJob<P>* jobs, int njob) {
    using R = typename PT<P>::R;
    const int bid = blockIdx.x;
    int jb = 0;
    while (jb + 1 < njob && bid >= jobs[jb + 1].blk0) ++jb;
    const BiVecJob<P>& J = jobs[jb];
    const int lb = bid - J.blk0;
    const int r = lb / J.nsb;
    const int sb = lb - r * J.nsb;
    const int cb = sb * VEC_BS + (int)threadIdx.x;
    const bool act = rhs_active(J, r);  // uniform over the block
    constexpr int NQ = (MODE == BV_RR || MODE == BV_RV || MODE == BV_SH) ? 2
                       : ((MODE == BV_TS || MODE == BV_XR) ? 3 : (MODE == BV_XRP ? 1 : 0));
    double* part = MODE == BV_SH ? J.part_s : J.part;
    if (!act) {  // the whole block: zero partials, no block sums
        if ((int)threadIdx.x < NQ) part[((long)r * NQ + (int)threadIdx.x) * J.pstride + sb] = 0.0;
        return;
    }
    double q0 = 0, q1 = 0, q2 = 0;
    if constexpr (P == P16 && (MODE == BV_S || MODE == BV_XR || MODE == BV_P || MODE == BV_SH || MODE == BV_XRP)) {
        // first pass: beyond the reach of the outputs everything is zero and stays so
        constexpr int reach = MODE == BV_SH ? 3 : 5;
        const bool near = (MODE != BV_SH && MODE != BV_XRP) || cb >= J.Vh ||
                          in_reach(J.tdist, J.titer, J.T, r, J.tdist ? cb / J.vt : 0, reach);
        if (act && near && cb < J.Vh) bivec16<MODE>(J, r, (uint32_t)cb, q0, q1, q2);
    } else if constexpr (MODE == BV_SH || MODE == BV_XRP) {
        // the merged iteration exists for FP16 fields only (launch_bivec refuses the others)
    } else if (act && cb < J.Vh) {
        R a[24], b[24], c[24];
        if (MODE == BV_RR || MODE == BV_RV) {
            load_spinor<P, R>(J.rh, J.Vh, r, cb, a);
            load_spinor<P, R>(MODE == BV_RR ? J.r : J.v, J.Vh, r, cb, b);
            for (int i = 0; i < 12; ++i) {
                const double ar = a[2 * i], ai = a[2 * i + 1], br = b[2 * i], bi = b[2 * i + 1];
                q0 += ar * br + ai * bi;
                q1 += ar * bi - ai * br;
            }
        } else if (MODE == BV_S) {
            const Cd al = ld2(J.alpha, r);
            load_spinor<P, R>(J.r, J.Vh, r, cb, a);
            load_spinor<P, R>(J.v, J.Vh, r, cb, b);
            for (int i = 0; i < 12; ++i) {
                const double br = b[2 * i], bi = b[2 * i + 1];
                c[2 * i] = (R)((double)a[2 * i] - (al.r * br - al.i * bi));
                c[2 * i + 1] = (R)((double)a[2 * i + 1] - (al.r * bi + al.i * br));
            }
            store_spinor<P, R>(J.s, J.Vh, r, cb, c);
        } else if (MODE == BV_TS) {
            load_spinor<P, R>(J.t, J.Vh, r, cb, a);
            load_spinor<P, R>(J.s, J.Vh, r, cb, b);
            for (int i = 0; i < 12; ++i) {
                const double ar = a[2 * i], ai = a[2 * i + 1], br = b[2 * i], bi = b[2 * i + 1];
                q0 += ar * br + ai * bi;
                q1 += ar * bi - ai * br;
                q2 += ar * ar + ai * ai;
            }
        } else if (MODE == BV_XR) {
            const Cd al = ld2(J.alpha, r), om = ld2(J.omega, r);
            load_spinor<P, R>(J.x, J.Vh, r, cb, a);
            load_spinor<P, R>(J.p, J.Vh, r, cb, b);
            load_spinor<P, R>(J.s, J.Vh, r, cb, c);
            for (int i = 0; i < 12; ++i) {
                const double pr = b[2 * i], pi = b[2 * i + 1], sr = c[2 * i], si = c[2 * i + 1];
                a[2 * i] = (R)((double)a[2 * i] + al.r * pr - al.i * pi + om.r * sr - om.i * si);
                a[2 * i + 1] = (R)((double)a[2 * i + 1] + al.r * pi + al.i * pr + om.r * si + om.i * sr);
            }
            store_spinor<P, R>(J.x, J.Vh, r, cb, a);
            load_spinor<P, R>(J.t, J.Vh, r, cb, b);
            for (int i = 0; i < 12; ++i) {
                const double tr = b[2 * i], ti = b[2 * i + 1];
                c[2 * i] = (R)((double)c[2 * i] - (om.r * tr - om.i * ti));
                c[2 * i + 1] = (R)((double)c[2 * i + 1] - (om.r * ti + om.i * tr));
            }
            store_spinor<P, R>(J.r, J.Vh, r, cb, c);
            // |r|^2 and (rh, r) of the new residual before its storage rounding
            load_spinor<P, R>(J.rh, J.Vh, r, cb, a);
            for (int i = 0; i < 12; ++i) {
                const double hr = a[2 * i], hi = a[2 * i + 1], rr = c[2 * i], ri = c[2 * i + 1];
                q0 += rr * rr + ri * ri;
                q1 += hr * rr + hi * ri;
                q2 += hr * ri - hi * rr;
            }
        } else {  // BV_P
            const Cd be = ld2(J.beta, r), om = ld2(J.omega, r);
            load_spinor<P, R>(J.r, J.Vh, r, cb, a);
            load_spinor<P, R>(J.p, J.Vh, r, cb, b);
            load_spinor<P, R>(J.v, J.Vh, r, cb, c);
            for (int i = 0; i < 12; ++i) {
                const double dr = (double)b[2 * i] - (om.r * c[2 * i] - om.i * c[2 * i + 1]);
                const double di = (double)b[2 * i + 1] - (om.r * c[2 * i + 1] + om.i * c[2 * i]);
                b[2 * i] = (R)((double)a[2 * i] + be.r * dr - be.i * di);
                b[2 * i + 1] = (R)((double)a[2 * i + 1] + be.r * di + be.i * dr);
            }
            store_spinor<P, R>(J.p, J.Vh, r, cb, b);
        }
    }
    if (NQ > 0) bi_partial(q0, part, ((long)r * NQ + 0) * J.pstride + sb);
    if (NQ > 1) bi_partial(q1, part, ((long)r * NQ + 1) * J.pstride + sb);
    if (NQ > 2) bi_partial(q2, part, ((long)r * NQ + 2) * J.pstride + sb);
}

template <int P> hipError_t launch_bivec(const BiVecJob<P>* j, int njob, int nblocks, int mode, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    switch (mode) {
    case BV_RR: hipLaunchKernelGGL((k_bivec<P, BV_RR>), dim3(nblocks), dim3(VEC_BS), 0, s, j, njob); break;
    case BV_RV: hipLaunchKernelGGL((k_bivec<P, BV_RV>), dim3(nblocks), dim3(VEC_BS), 0, s, j, njob); break;
    case BV_S: hipLaunchKernelGGL((k_bivec<P, BV_S>), dim3(nblocks), dim3(VEC_BS), 0, s, j, njob); break;
    case BV_TS: hipLaunchKernelGGL((k_bivec<P, BV_TS>), dim3(nblocks), dim3(VEC_BS), 0, s, j, njob); break;
    case BV_XR: hipLaunchKernelGGL((k_bivec<P, BV_XR>), dim3(nblocks), dim3(VEC_BS), 0, s, j, njob); break;
    case BV_P: hipLaunchKernelGGL((k_bivec<P, BV_P>), dim3(nblocks), dim3(VEC_BS), 0, s, j, njob); break;
    case BV_SH:
        if (P != P16) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_bivec<P, BV_SH>), dim3(nblocks), dim3(VEC_BS), 0, s, j, njob);
        break;
    case BV_XRP:
        if (P != P16) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_bivec<P, BV_XRP>), dim3(nblocks), dim3(VEC_BS), 0, s, j, njob);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template hipError_t launch_bivec<P64>(const BiVecJob<P64>*, int, int, int, hipStream_t);
template hipError_t launch_bivec<P32>(const BiVecJob<P32>*, int, int, int, hipStream_t);
template hipError_t launch_bivec<P16>(const BiVecJob<P16>*, int, int, int, hipStream_t);
template hipError_t launch_bivec<PB16>(const BiVecJob<PB16>*, int, int, int, hipStream_t);

// One block per right-hand side: fixed-order sums of the quantities' partials, then
// the scalar update of the mode.  A right-hand side stops (inactive) when |r|^2
// reaches its target, at the iteration cap, on a non-finite value, or on a
// breakdown (a zero denominator); the defect-correction pass that runs the inner
// solve restarts from the true residual in every case.
__global__ void __launch_bounds__(256) k_bifinish(const BiFinJob* jobs, int njob, int mode) {
    const int bid = blockIdx.x;
    int jb = 0;
    while (jb + 1 < njob && bid >= jobs[jb + 1].rhs0) ++jb;
    const BiFinJob& J = jobs[jb];
    const int r = bid - J.rhs0;
    if (r >= J.nrhs) return;  // uniform over the block
    const int NQ = (mode == BF_ALPHA || mode == BF_INIT) ? 2 : (mode == BF_OMBETA ? 5 : (mode == BF_CONV ? 1 : 3));
    const int np = (mode == BF_ALPHA || mode == BF_OMEGA || mode == BF_OMBETA) ? J.nparth : J.npart;
    __shared__ double lds[4];
    double q[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < NQ; ++k) {
        double v = 0;
        const double* pp = J.part + ((size_t)r * NQ + k) * np;
        for (int i = threadIdx.x; i < np; i += 256) v += pp[i];
        q[k] = block_sum<256>(v, lds);
    }
    if (mode == BF_OMBETA)  // (rh, s) from the s step's own partials
        for (int k = 0; k < 2; ++k) {
            double v = 0;
            const double* pp = J.part_s + ((size_t)r * 2 + k) * J.npart;
            for (int i = threadIdx.x; i < J.npart; i += 256) v += pp[i];
            q[5 + k] = block_sum<256>(v, lds);
        }
    if (threadIdx.x != 0) return;
    const Cd one = {1.0, 0.0}, zero = {0.0, 0.0};
    auto st = [](double2* a, int i, Cd v) { a[i] = make_double2(v.r, v.i); };
    if (mode == BF_INIT) {  // start of an inner solve (after the CG-state init): rho = (rh, r)
        const Cd rho = {q[0], q[1]};
        st(J.rho, r, rho);
        st(J.alpha, r, one);
        st(J.omega, r, one);
        st(J.beta, r, zero);
        if (J.active[r] && (!finite2(rho) || (rho.r == 0.0 && rho.i == 0.0))) J.active[r] = 0;
        return;
    }
    if (!J.active[r]) return;
    if (mode == BF_ALPHA) {
        const Cd d = {q[0], q[1]};
        if (!finite2(d) || (d.r == 0.0 && d.i == 0.0)) {
            st(J.alpha, r, zero);
            J.active[r] = 0;
        } else {
            st(J.alpha, r, cdivc(ld2(J.rho, r), d));
        }
    } else if (mode == BF_OMEGA) {
        const Cd ts = {q[0], q[1]};
        st(J.omega, r, (finite2(ts) && q[2] > 0.0 && isfinite(q[2])) ? Cd{ts.r / q[2], ts.i / q[2]} : zero);
    } else if (mode == BF_OMBETA) {
        // omega = (t, s) / |t|^2; rho' = (rh, s) - omega (rh, t), both on the stored s and t, is
        // (rh, s - omega t) for the r = s - omega t that the merged update forms from them
        const Cd ts = {q[0], q[1]}, rt = {q[3], q[4]}, rs = {q[5], q[6]};
        const Cd om = (finite2(ts) && q[2] > 0.0 && isfinite(q[2])) ? Cd{ts.r / q[2], ts.i / q[2]} : zero;
        st(J.omega, r, om);
        const Cd ort = cmulc(om, rt);
        const Cd rho1 = {rs.r - ort.r, rs.i - ort.i};
        const Cd rho = ld2(J.rho, r), al = ld2(J.alpha, r);
        const bool brk = (om.r == 0.0 && om.i == 0.0) || (rho.r == 0.0 && rho.i == 0.0) || !finite2(rho1) ||
                         (rho1.r == 0.0 && rho1.i == 0.0);
        // on a breakdown the update still runs (with beta = 0) and BF_CONV stops the right-hand side
        st(J.beta, r, brk ? zero : cmulc(cdivc(rho1, rho), cdivc(al, om)));
        st(J.rho, r, brk ? zero : rho1);
    } else if (mode == BF_CONV) {
        const double rr = q[0];
        J.rr[r] = rr;
        const int it = J.iters[r] + 1;
        J.iters[r] = it;
        const Cd rho = ld2(J.rho, r);  // zero after a breakdown
        if (!isfinite(rr) || rr <= J.tol2[r] || it >= J.maxit || (rho.r == 0.0 && rho.i == 0.0)) J.active[r] = 0;
    } else {  // BF_BETA
        const double rr = q[0];
        const Cd rho1 = {q[1], q[2]};
        J.rr[r] = rr;
        const int it = J.iters[r] + 1;
        J.iters[r] = it;
        const Cd rho = ld2(J.rho, r), om = ld2(J.omega, r), al = ld2(J.alpha, r);
        const bool brk = (om.r == 0.0 && om.i == 0.0) || (rho.r == 0.0 && rho.i == 0.0) || !finite2(rho1);
        if (!isfinite(rr) || rr <= J.tol2[r] || it >= J.maxit || brk) {
            J.active[r] = 0;
            return;
        }
        st(J.beta, r, cmulc(cdivc(rho1, rho), cdivc(al, om)));
        st(J.rho, r, rho1);
    }
}

hipError_t launch_bifinish(const BiFinJob* j, int njob, int nblocks, int mode, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bifinish, dim3(nblocks), dim3(256), 0, s, j, njob, mode);
    return hipGetLastError();
}

}  // namespace dlma
