// Even-odd Wilson-clover stencil kernels, multi right-hand side.
//
// With H_pq the hopping sum from parity q to parity p,
//   (H psi)(x) = sum_mu [(1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu)],
// the operator is D = A - H/2, and the Schur complement on even sites is
//   Dhat = A_ee - (1/4) H_eo A_oo^-1 H_oe,  Dhat^dag = g5 Dhat g5.
// Two kernel kinds cover every use:
//   K1 (output parity p):  out = A_pp^-1 (d + ch * H [g5] in)            [+= out with ACCUM]
//   K2 (output parity p):  out = cb*b + ca*(A_pp x) + ch * [g5] H in     [A -> 1 with NOA]
// with optional fused epilogues: per-RHS squared norms of the result (NORM) and
// the CG update r -= alpha*out, xs += alpha*x (CG; out itself is not stored).
//
// Thread mapping: one thread per output site and NB right-hand sides; a block
// covers BS consecutive sites for one group of NB right-hand sides.  The block
// index is decoded so that all right-hand-side groups of one site block land on
// the same XCD (workgroups are dealt round-robin to the 8 XCDs) one after the
// other, so the links and clover of that site block are reused from that XCD's L2,
// and each XCD sweeps a contiguous range of site blocks so that neighbour spinors
// loaded for one block are still in its L2 for the next.
#pragma once
#include "common.h"

namespace dlma {

enum HopKind { K1 = 0, K2 = 1 };
enum HopFlags {
    F_G5IN = 1,     // K1: g5 on the hopping input
    F_G5OUT = 2,    // K2: g5 on the hopping sum
    F_NORM = 4,     // per-RHS |out|^2 partials
    F_CG = 8,       // K2: r -= alpha*out, xs += alpha*x, |r|^2 partials; out not stored
    F_HASB = 16,    // K2: add cb*b
    F_NOA = 32,     // K2: identity instead of the clover matrix
    F_HASD = 64,    // K1: add d (taken from the x view)
    F_ACCUM = 128,  // K1: out += result
    F_DOTX = 256,   // K2: partials of sum conj(out) x (re, im) and |out|^2
    F_DOTR = 512,   // K2: partials of sum conj(r) out (re, im), r the job's r field
    F_DOTXH = 1024, // K2, FP16, with F_DOTX: also sum conj(r) out of the stored (rounded) out (re, im)
    F_IN16 = 2048,  // FP64 kernels: the hopping input is the FP16 field in16 times sqrt(in16s[r])
    F_ACCX = 4096,  // K2, FP64: first x += in16 * sqrt(in16s[r]) (stored), then the operator on it
};

// Partial sums a stencil launch writes per right-hand side: F_DOTX | F_DOTXH 5,
// F_DOTX 3, F_DOTR 2, F_NORM or F_CG 1 (|out|^2 or the updated |r|^2).  Layout: one
// quantity at part[r * pstride + block]; several at part[(r * NQ + q) * pstride + block].
constexpr int hop_nq(int fl) {
    return (fl & F_DOTXH) ? 5 : ((fl & F_DOTX) ? 3 : ((fl & F_DOTR) ? 2 : ((fl & (F_NORM | F_CG)) ? 1 : 0)));
}
constexpr int HOP_NQ_MAX = 5;

template <int P> struct HopJob {
    Geo g;
    int par;    // output parity
    int nrhs;   // right-hand sides
    int G;      // right-hand-side groups = ceil(nrhs / NB)
    int vt;     // sites of one parity on one timeslice (Z*Y*X/2)
    int nbt;    // site blocks per timeslice = ceil(vt / BS); a block never spans two timeslices
    int nsb;    // site blocks = T * nbt
    int nxb;    // site blocks per XCD = ceil(T/8) * nbt
    int blk0;   // first workgroup of this job (multiple of 8)
    int sg;     // right-hand-side groups per super-group (see the block decode); 0 = all groups
    const typename PT<P>::S* U;  // links, all parities
    const typename PT<P>::S* C;  // clover blocks of the output parity (A or A^-1)
    SF<P> in, x, b, out, r, xs;
    SF<P16> in16;         // F_IN16: hopping input in FP16 storage (grouped words, site scales)
    const double* in16s;  // F_IN16: [nrhs] squared factor of in16
    // FP64 kernels: timeslice support flags [nrhs][T] of the source B (see VecJob) or
    // nullptr.  Jobs that read B skip it where it vanishes: b (F_HASB) and d (F_HASD)
    // on unflagged timeslices, and the pass-0 Schur source (F_NOA, from B_e and
    // A_oo^-1 B_o) is zero where t - 1 .. t + 1 are all unflagged.
    const int* tsup;
    const double* alpha;  // [nrhs] (F_CG)
    const int* active;    // [nrhs] or nullptr: inactive right-hand sides are skipped
    double* part;         // partial squared norms (F_NORM / F_CG): part[r * pstride + site block]
    int pstride;
    int wn;     // FP16 stencils: sites in the block's LDS window of +-x, +-y neighbours (0 = none)
    double ca, cb, ch;
};

// A value the caller knows to be the same on every lane, marked as such so that
// branches on it and values merged after them stay in scalar registers.
HD int wave_uniform(int v) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_readfirstlane(v);
#else
    return v;
#endif
}

// Whether right-hand side r of job J is still iterating.  Every branch here is on
// a wave-uniform value (the flag is read once and marked uniform), so the values
// that meet after it (field addresses, buffer resources) stay in scalar registers.
template <class Job> HD bool rhs_active(const Job& J, int r) {
    if (r >= J.nrhs) return false;
    if (J.active == nullptr) return true;
    return wave_uniform(J.active[r]) != 0;
}

template <int P, class R> HD void load_half_spinor(const SF<P>& f, int Vh, int r, int cb, int blk, R s[12]) {
    static_assert(P != P16, "FP16 fields use the grouped layout of hop16.h");
    const typename PT<P>::S* b = f.v + (size_t)r * f.rs + (size_t)blk * 6 * Vh + cb;
#pragma unroll
    for (int c = 0; c < 6; ++c) ldp<P>(b, (size_t)c * Vh, s[2 * c], s[2 * c + 1]);
    if (P == P16) {
        R n = (R)f.nrm[(size_t)r * f.ns + cb];
#pragma unroll
        for (int i = 0; i < 12; ++i) s[i] *= n;
    }
}

template <int P, class R> HD void store_half_spinor(const SF<P>& f, int Vh, int r, int cb, int blk, const R s[12]) {
    static_assert(P != P16, "FP16 fields use the grouped layout of hop16.h");
    typename PT<P>::S* b = f.v + (size_t)r * f.rs + (size_t)blk * 6 * Vh + cb;
#pragma unroll
    for (int c = 0; c < 6; ++c) stp<P>(b, (size_t)c * Vh, (typename PT<P>::R)s[2 * c], (typename PT<P>::R)s[2 * c + 1]);
}

// The hopping input of right-hand side r at site cb: the job's field, or with IN16
// (FP64 kernels) the FP16 field in16 times fac.
template <int P, bool IN16, class R>
HD void load_input(const HopJob<P>& J, int Vh, int r, int cb, double fac, R psi[24]) {
    if constexpr (IN16 && P == P64) load_spinor16_f64(J.in16, Vh, r, cb, fac, psi);
    else load_spinor<P, R>(J.in, Vh, r, cb, psi);
}

template <int P, int NB, int MU, bool G5IN, bool IN16>
HD void hop_dir(const HopJob<P>& J, const Nbr& nb, int cb, int g0, bool (&use)[NB], const double (&fac)[NB],
                typename PT<P>::R (&acc)[NB][24]) {
    using R = typename PT<P>::R;
    const int Vh = J.g.Vh;
    R u[18];
    R psi[24];
    load_link<P, R>(J.U, Vh, J.par, MU, cb, u);
#pragma unroll
    for (int j = 0; j < NB; ++j)
        if (use[j]) {
            load_input<P, IN16, R>(J, Vh, g0 + j, nb.n[2 * MU], fac[j], psi);
            hop_term<MU, true, G5IN, R>(u, psi, acc[j]);
        }
    load_link<P, R>(J.U, Vh, 1 - J.par, MU, nb.n[2 * MU + 1], u);
#pragma unroll
    for (int j = 0; j < NB; ++j)
        if (use[j]) {
            load_input<P, IN16, R>(J, Vh, g0 + j, nb.n[2 * MU + 1], fac[j], psi);
            hop_term<MU, false, G5IN, R>(u, psi, acc[j]);
        }
}

// Per-site body.  Returns the site's contributions to the partial sums of hop_nq(FL)
// quantities in qs.
template <int P, int NB, int KIND, int FL>
HD void hop_site(const HopJob<P>& J, int cb, int g0, double (&qs)[NB][HOP_NQ_MAX]) {
    static_assert(P != P16, "FP16 fields take hop_site16");
    using R = typename PT<P>::R;
    const int Vh = J.g.Vh;
    bool use[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        int r = g0 + j;
        use[j] = rhs_active(J, r);
        for (int q = 0; q < HOP_NQ_MAX; ++q) qs[j][q] = 0.0;
    }
    R acc[NB][24];
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int i = 0; i < 24; ++i) acc[j][i] = 0;
    // timeslice of the site (uniform over the block) for the source-support tests
    const int tsite = J.tsup ? cb / J.vt : 0;
    if constexpr (KIND == K2 && (FL & F_NOA) != 0) {
        // Schur source of a source that vanishes on t - 1 .. t + 1: zero, nothing to load
        if (J.tsup) {
            bool any = false;
#pragma unroll
            for (int j = 0; j < NB; ++j) any = any || (use[j] && tsup_any(J.tsup, J.g.T, g0 + j, tsite, 1));
            if (!any) {
#pragma unroll
                for (int j = 0; j < NB; ++j)
                    if (use[j]) store_spinor<P, R>(J.out, Vh, g0 + j, cb, acc[j]);
                return;
            }
        }
    }

    Nbr nb = neighbours(J.g, J.par, cb);
    constexpr bool G5IN = (FL & F_G5IN) != 0;
    constexpr bool IN16 = (FL & F_IN16) != 0;
    static_assert(!IN16 || P == P64, "an FP16 hopping input is for the FP64 kernels");
    double fac[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) fac[j] = (IN16 && use[j]) ? sqrt(J.in16s[g0 + j]) : 1.0;
    hop_dir<P, NB, 0, G5IN, IN16>(J, nb, cb, g0, use, fac, acc);
    hop_dir<P, NB, 1, G5IN, IN16>(J, nb, cb, g0, use, fac, acc);
    hop_dir<P, NB, 2, G5IN, IN16>(J, nb, cb, g0, use, fac, acc);
    hop_dir<P, NB, 3, G5IN, IN16>(J, nb, cb, g0, use, fac, acc);

    const R ch = (R)J.ch;
    if (KIND == K1) {
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (use[j]) {
#pragma unroll
                for (int i = 0; i < 24; ++i) acc[j][i] *= ch;
                if ((FL & F_HASD) && tsup_any(J.tsup, J.g.T, g0 + j, tsite, 0)) {
                    R d[24];
                    load_spinor<P, R>(J.x, Vh, g0 + j, cb, d);
#pragma unroll
                    for (int i = 0; i < 24; ++i) acc[j][i] += d[i];
                }
            }
#pragma unroll
        for (int blk = 0; blk < 2; ++blk) {
            R c[36];
            load_clover_block<P, R>(J.C, Vh, blk, cb, c);
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (use[j]) {
                    R t[12];
                    herm6<R>(c, &acc[j][blk * 12], t);
#pragma unroll
                    for (int i = 0; i < 12; ++i) acc[j][blk * 12 + i] = t[i];
                }
        }
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (use[j]) {
                if (FL & F_ACCUM) {
                    R o[24];
                    load_spinor<P, R>(J.out, Vh, g0 + j, cb, o);
#pragma unroll
                    for (int i = 0; i < 24; ++i) acc[j][i] += o[i];
                }
                store_spinor<P, R>(J.out, Vh, g0 + j, cb, acc[j]);
                if (FL & F_NORM) {
                    double s = 0;
#pragma unroll
                    for (int i = 0; i < 24; ++i) s += (double)acc[j][i] * (double)acc[j][i];
                    qs[j][0] = s;
                }
            }
    } else {
        const R ca = (R)J.ca;
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (use[j]) {
#pragma unroll
                for (int i = 0; i < 24; ++i) acc[j][i] *= ch;
                if (FL & F_G5OUT) {
#pragma unroll
                    for (int i = 12; i < 24; ++i) acc[j][i] = -acc[j][i];
                }
            }
        // F_ACCX: the correction of the last inner solve is added to x here (the even
        // sites' accumulation of the defect correction, fused into the next residual)
        constexpr bool ACCX = (FL & F_ACCX) != 0;
        static_assert(!ACCX || P == P64, "the fused accumulation is for the FP64 residual");
        double facx[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) facx[j] = (ACCX && use[j]) ? sqrt(J.in16s[g0 + j]) : 0.0;
#pragma unroll
        for (int blk = 0; blk < 2; ++blk) {
            R c[36];
            if (!(FL & F_NOA)) load_clover_block<P, R>(J.C, Vh, blk, cb, c);
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (use[j]) {
                    R xv[12], t[12];
                    load_half_spinor<P, R>(J.x, Vh, g0 + j, cb, blk, xv);
                    if constexpr (ACCX && P == P64) {
                        add_half16_f64(J.in16, Vh, g0 + j, cb, blk, facx[j], xv);
                        store_half_spinor<P, R>(J.x, Vh, g0 + j, cb, blk, xv);
                    }
                    if (FL & F_NOA) {
#pragma unroll
                        for (int i = 0; i < 12; ++i) t[i] = xv[i];
                    } else {
                        herm6<R>(c, xv, t);
                    }
#pragma unroll
                    for (int i = 0; i < 12; ++i) acc[j][blk * 12 + i] += ca * t[i];
                }
        }
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (use[j]) {
                if ((FL & F_HASB) && tsup_any(J.tsup, J.g.T, g0 + j, tsite, 0)) {
                    R bv[24];
                    load_spinor<P, R>(J.b, Vh, g0 + j, cb, bv);
                    const R cbc = (R)J.cb;
#pragma unroll
                    for (int i = 0; i < 24; ++i) acc[j][i] += cbc * bv[i];
                }
                if (FL & F_CG) {
                    const R al = (R)J.alpha[g0 + j];
                    R rv[24], w[24];
                    load_spinor<P, R>(J.r, Vh, g0 + j, cb, rv);
#pragma unroll
                    for (int i = 0; i < 24; ++i) rv[i] -= al * acc[j][i];
                    store_spinor<P, R>(J.r, Vh, g0 + j, cb, rv);
                    double s = 0;
#pragma unroll
                    for (int i = 0; i < 24; ++i) s += (double)rv[i] * (double)rv[i];
                    qs[j][0] = s;
                    load_spinor<P, R>(J.x, Vh, g0 + j, cb, w);
                    load_spinor<P, R>(J.xs, Vh, g0 + j, cb, rv);
#pragma unroll
                    for (int i = 0; i < 24; ++i) rv[i] += al * w[i];
                    store_spinor<P, R>(J.xs, Vh, g0 + j, cb, rv);
                } else {
                    store_spinor<P, R>(J.out, Vh, g0 + j, cb, acc[j]);
                    if (FL & (F_NORM | F_DOTX)) {
                        double s = 0;
#pragma unroll
                        for (int i = 0; i < 24; ++i) s += (double)acc[j][i] * (double)acc[j][i];
                        qs[j][(FL & F_DOTX) ? 2 : 0] = s;
                    }
                    if (FL & (F_DOTX | F_DOTR)) {
                        R v[24];
                        if (FL & F_DOTX) load_spinor<P, R>(J.x, Vh, g0 + j, cb, v);
                        else load_spinor<P, R>(J.r, Vh, g0 + j, cb, v);
                        double re = 0, im = 0;
#pragma unroll
                        for (int c = 0; c < 12; ++c) {
                            // F_DOTX: conj(out) x; F_DOTR: conj(r) out
                            const double ar = (FL & F_DOTX) ? acc[j][2 * c] : v[2 * c];
                            const double ai = (FL & F_DOTX) ? acc[j][2 * c + 1] : v[2 * c + 1];
                            const double br = (FL & F_DOTX) ? v[2 * c] : acc[j][2 * c];
                            const double bi = (FL & F_DOTX) ? v[2 * c + 1] : acc[j][2 * c + 1];
                            re += ar * br + ai * bi;
                            im += ar * bi - ai * br;
                        }
                        qs[j][0] = re;
                        qs[j][1] = im;
                    }
                }
            }
    }
}

}  // namespace dlma

#include "hop16.h"

namespace dlma {

// ---------------------------------------------------------------- block reduction

// Sum of v over the block (BS threads, wave64), result valid in thread 0.
template <int BS> __device__ __forceinline__ double block_sum(double v, double* lds) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    constexpr int NW = BS / 64;
    if (NW == 1) return v;
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NW; ++i) s += lds[i];
    __syncthreads();
    return s;
}

// The per-site body for the FP64, FP32 and BF16 fields (FP16 fields take the
// raw-word path of hop16.h, called from the kernel directly).
template <int P, int NB, int KIND, int FL>
HD void site_body(const HopJob<P>& J, int cb, int g0, double (&qs)[NB][HOP_NQ_MAX]) {
    hop_site<P, NB, KIND, FL>(J, cb, g0, qs);
}

// Occupancy floor per instantiation: the FP16 kernels with up to two right-hand
// sides per thread stay within 128 registers (four waves per SIMD), which their
// long-latency gathers need; the compiler's own choice lands just above it for some.
template <int P, int NB> constexpr int hop_min_waves() { return (P == P16 && NB <= 2) ? 4 : 1; }

// wn_cap: window sites per right-hand side that the launch's dynamic LDS holds
// (NB * wn_cap * 52 bytes); a job stages its window only if it fits.
template <int P, int NB, int KIND, int FL, int BS>
__global__ void __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(hop_min_waves<P, NB>())))
hop_kernel(const HopJob<P>* __restrict__ jobs, int njob, int wn_cap, int tw0, int twn) {
    const int bid = blockIdx.x;
    int jb = 0;
    while (jb + 1 < njob && bid >= jobs[jb + 1].blk0) ++jb;
    const HopJob<P>& J = jobs[jb];
    // Block decode.  Workgroups are dealt round-robin to the 8 XCDs, so XCD (lb & 7)
    // runs the sequence k = lb >> 3.  Each XCD owns a contiguous range of timeslices.
    // Its sequence runs over super-groups of SG right-hand-side groups; within one
    // super-group it walks the site blocks of a timeslice (index s) in the outer loop,
    // its timeslices in the middle loop and the SG groups innermost.  A block's links
    // and clover are then reused by the SG groups straight away, its +-t neighbours
    // were loaded SG blocks earlier, and its +-z neighbours about 2*(Z*Y*X/2)/BS * nt * SG
    // blocks earlier (nt = timeslices per XCD): small SG keeps those halos in the XCD's
    // L2, large SG reads the links and clover fewer times.
    const int lb = bid - J.blk0;
    const int xcd = lb & 7;
    const int k = lb >> 3;
    const int T = J.g.T;
    // the launch covers every timeslice (twn = 0) or the window tw0 .. tw0 + twn - 1
    // (periodic; one job only): a first-pass launch whose input vanishes elsewhere
    const int Tw = twn > 0 ? twn : T;
    const int tl = xcd * Tw / 8, nt = (xcd + 1) * Tw / 8 - tl;
    if (nt == 0) return;  // more XCDs than timeslices
    const int SG = (J.sg > 0 && J.sg < J.G) ? J.sg : J.G;
    const int per = J.nbt * nt * SG;
    const int si = k / per;
    if (si * SG >= J.G) return;  // padding of the XCD decomposition
    const int kk = k - si * per;
    const int sge = min(SG, J.G - si * SG);
    if (kk >= J.nbt * nt * sge) return;
    const int q = kk / sge;
    const int gi = si * SG + (kk - q * sge);
    const int s = q / nt;
    const int tw = tl + (q - s * nt);
    const int t = twn > 0 ? (tw0 + tw < T ? tw0 + tw : tw0 + tw - T) : tw;
    const int sb = t * J.nbt + s;
    const int sx = s * BS + (int)threadIdx.x;  // site within the timeslice
    const int cb = t * J.vt + sx;
    const int g0 = gi * NB;
    // right-hand-side groups with nothing active skip the block (partials written as 0)
    bool live = false;
#pragma unroll
    for (int j = 0; j < NB; ++j) live = live || rhs_active(J, g0 + j);
    constexpr int NQ = hop_nq(FL);
    if (!live) {
        if (NQ > 0 && (int)threadIdx.x < NB * NQ && g0 + (int)threadIdx.x / NQ < J.nrhs)
            J.part[(size_t)(g0 * NQ + (int)threadIdx.x) * J.pstride + sb] = 0.0;
        return;
    }
    double qs[NB][HOP_NQ_MAX];
    if constexpr (P == P16) {
        // Every thread runs the body, whose LDS staging has a block barrier: a thread
        // past the timeslice's last site works on that site and stores nothing.
        extern __shared__ __attribute__((aligned(16))) uint32_t hop_window[];
        const bool valid = sx < J.vt;
        const int ts0 = t * J.vt;
        const int wn = (J.wn > 0 && J.wn <= wn_cap) ? J.wn : 0;
        const Window16 win{wn, ts0 + s * BS - J.g.Xh, ts0, ts0 + J.vt, (LdsWords)hop_window};
        hop_site16<NB, KIND, FL, BS>(J, valid ? cb : ts0 + J.vt - 1, g0, valid, win, qs);
    } else {
        if (sx < J.vt) {
            site_body<P, NB, KIND, FL>(J, cb, g0, qs);
        } else {
#pragma unroll
            for (int j = 0; j < NB; ++j)
                for (int q = 0; q < HOP_NQ_MAX; ++q) qs[j][q] = 0.0;
        }
    }
    if (NQ > 0) {
        __shared__ double lds[BS / 64];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (g0 + j >= J.nrhs) break;  // uniform over the block
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                double s = block_sum<BS>(qs[j][q], lds);
                if (threadIdx.x == 0) J.part[((size_t)(g0 + j) * NQ + q) * J.pstride + sb] = s;
            }
        }
    }
}

}  // namespace dlma
