// Launch descriptors and host-side launchers of the dlma kernels.
#pragma once
#include "hop.h"

namespace dlma {

// Site-local vector kernels over half-lattice fields (one thread per site and
// right-hand side), batched over jobs like the stencil kernels.
template <int P> struct VecJob {
    int Vh, nrhs, nsb, blk0;  // nsb = ceil(Vh / VEC_BS); blocks of the job = nsb * nrhs
    SF<P> a, b, c;
    const double2* C;     // clover blocks (clover apply)
    const double* s;      // per right-hand side scalar
    const int* active;    // per right-hand side flag or nullptr
    double* part;         // partial squared norms, row stride pstride
    int pstride;
    // Timeslice support of the source: flag [r][t] = 1 where source r has a nonzero
    // component on timeslice t (either parity).  k_norm records it (tsup_out); the
    // pass-0 kernels read it (tsup) and skip the loads of an input known to be zero:
    // the input vanishes on timeslice t when the flags of t - tdil .. t + tdil are all 0.
    int* tsup_out;
    const int* tsup;
    int tdil;
    int vt, T;            // sites of one parity per timeslice, timeslices
};
constexpr int VEC_BS = 256;

// Per right-hand side finishing of two-stage reductions (one block per rhs, fixed order).
struct FinJob {
    int nrhs, rhs0, npart;     // rhs0: first global block of this job
    const double* part;        // [nrhs][npart]
    double* rr;                // CG: current |r|^2
    double* rr0;               // CG: |r|^2 at start
    double* alpha;
    double* beta;
    double* tol2;              // CG: stop when |r|^2 <= tol2 (set by FIN_INIT)
    const double* abs2;        // FIN_INIT: absolute target of |r|^2
    double rel2;               // FIN_INIT: relative target, tol2 = max(rel2 * |r0|^2, abs2)
    int* active;
    int* iters;
    int maxit;
    double* out;               // FIN_NORM: sums; FIN_INIT: |bhat|^2 (scale of the unit-norm inner source)
};
enum FinMode { FIN_NORM = 0, FIN_ALPHA = 1, FIN_BETA = 2, FIN_INIT = 3 };

// BiCGStab on the even-odd reduced operator (the alternative inner solver).  Site-
// local vector steps, one thread per site and right-hand side; partial sums of NQ
// quantities per block at part[(r * NQ + q) * pstride + site block].
template <int P> struct BiVecJob {
    int Vh, nrhs, nsb, blk0;
    SF<P> r, rh, p, v, s, t, x;        // residual, shadow residual, direction, D p, s, D s, iterate
    const double2 *alpha, *omega, *beta;  // per right-hand side
    const int* active;
    double* part;
    int pstride;
    double* part_s;  // BV_SH's partials of (rh, s), part_s[(r * 2 + q) * pstride + block] (FP16 path)
    // first pass, FP16: sites beyond the reach of the step's outputs (in_reach; s: 3,
    // x/r/p: 5) are skipped; vt = sites of one parity per timeslice
    const int* tdist;
    const int* titer;
    int vt, T;
};
enum BiVecMode {
    BV_RR = 0,    // part: (rh, r)                                   NQ = 2 (re, im)
    BV_RV = 1,    // part: (rh, v)                                   NQ = 2 (re, im)
    BV_S = 2,     // s = r - alpha v
    BV_TS = 3,    // part: (t, s), |t|^2                             NQ = 3
    BV_XR = 4,    // x += alpha p + omega s; r = s - omega t; part: |r|^2, (rh, r)   NQ = 3
    BV_P = 5,     // p = r + beta (p - omega v)
    // FP16 fields only: the merged iteration (beta known before the updates)
    BV_SH = 6,    // s = r - alpha v; part_s: (rh, s) of the stored s  NQ = 2
    BV_XRP = 7,   // x += alpha p + omega s; r = s - omega t; p = r + beta (p - omega v); part: |r|^2  NQ = 1
};
template <int P> hipError_t launch_bivec(const BiVecJob<P>* j, int njob, int nblocks, int mode, hipStream_t s);

// Per right-hand side scalars of BiCGStab from the partial sums (one block per rhs,
// fixed order), with the CG state of FinJob (|r|^2, targets, flags, counts).
struct BiFinJob {
    int nrhs, rhs0, npart;     // npart: partials per quantity of the vector kernels (their pstride)
    int nparth;                // the same for the stencil kernels (alpha's and omega's sums come from K2)
    const double* part;
    const double* part_s;      // BV_SH's partials of (rh, s) (pstride npart)
    double2 *rho, *alpha, *omega, *beta;
    double *rr, *tol2;
    int *active, *iters;
    int maxit;
};
enum BiFinMode { BF_INIT = 0, BF_ALPHA = 1, BF_OMEGA = 2, BF_BETA = 3, BF_OMBETA = 4, BF_CONV = 5 };
// BF_ALPHA reads (rh, v) from K2 with F_DOTR, BF_OMEGA (t, s) and |t|^2 from K2 with
// F_DOTX (layout of hop_nq), BF_INIT and BF_BETA the vector kernels' sums.
// Merged iteration: BF_OMBETA reads (t, s), |t|^2 and (rh, t) from K2 with F_DOTX |
// F_DOTXH and (rh, s) from BV_SH, and forms omega, rho' = (rh, s) - omega (rh, t) =
// (rh, s - omega t) and beta before the updates; BF_CONV reads BV_XRP's |r|^2 and
// decides convergence and breakdown.
hipError_t launch_bifinish(const BiFinJob* j, int njob, int nblocks, int mode, hipStream_t s);

// wn: LDS window sites per right-hand side of the launch's FP16 jobs (the largest
// HopJob::wn among them; 0 = none, and always 0 for other precisions)
// wn: LDS window sites of the FP16 stencils.  tw0, twn: the launch covers timeslices
// tw0 .. tw0 + twn - 1 (periodic) of its single job; twn = 0: every timeslice (the
// block count is then that of assign_blocks, else hop_window_blocks).
struct HopCfg { int kind, flags, nb, wn = 0, tw0 = 0, twn = 0; };
constexpr int HOP_BS = 128;

// Dynamic LDS of an FP16 stencil launch: per right-hand side and window site, three
// 16-byte word groups and the 4-byte scale.
constexpr unsigned hop_window_bytes(int nb, int wn) { return (unsigned)(nb * wn * 52); }
// Largest dynamic LDS a stencil block may take: with up to two right-hand sides per
// thread, eight blocks of two waves (four waves per SIMD) share a CU's 160 KiB; with
// four, the registers allow two waves per SIMD and four blocks.
constexpr int hop_window_max_bytes(int nb) { return nb <= 2 ? 20 * 1024 : 40 * 1024; }

template <int P> hipError_t launch_hop(const HopCfg& c, const HopJob<P>* djobs, int njob, int nblocks, hipStream_t s);

// gauge and clover
hipError_t launch_pack_links(const double2* Ucan, double2* U64, const Geo& g, hipStream_t s);
hipError_t launch_unitarity(const double2* Ucan, long nlink, double* blockmax, int nblk, hipStream_t s);
hipError_t launch_clover_build(const double2* Ucan, const Geo& g, double m0, double csw, double2* C0, double2* C1, hipStream_t s);
hipError_t launch_clover_invert(const double2* C, double2* Ci, int Vh, int* err, hipStream_t s);
hipError_t launch_add_diag(double2* C, int Vh, double delta, hipStream_t s);
template <int P> hipError_t launch_convert_pairs(const double2* src, void* dst, long n, hipStream_t s);
hipError_t launch_regroup16(const double2* src, void* dst, int M, int K, int G, int Vh, hipStream_t s);

// full FP64 fields <-> canonical
hipError_t launch_canon_to_eo(const double2* can, double2* eo, const Geo& g, int nrhs, hipStream_t s, int g5 = 0);
hipError_t launch_eo_to_canon(const double2* eo, double2* can, const Geo& g, int nrhs, hipStream_t s, int g5 = 0);

// vector kernels (jobs in device memory, total blocks given)
hipError_t launch_clover_apply64(const VecJob<P64>* j, int njob, int nblocks, hipStream_t s);  // c = C a
// dist[r][t] = periodic distance from t to the nearest t' with flags[r][t'] != 0
// (2^28 if there is none), for nrhs x T entries
hipError_t launch_tdist(const int* flags, int* dist, int nrhs, int T, hipStream_t s);
template <int P> hipError_t launch_conv_from64(const VecJob<P>* j, int njob, int nblocks, const VecJob<P64>* j64, hipStream_t s);
template <int P> hipError_t launch_accum_to64(const VecJob<P>* j, const VecJob<P64>* j64, int njob, int nblocks, hipStream_t s);
template <int P> hipError_t launch_xpay(const VecJob<P>* j, int njob, int nblocks, hipStream_t s);       // b = a + s*b
template <int P> hipError_t launch_norm(const VecJob<P>* j, int njob, int nblocks, hipStream_t s);       // part = |a|^2
template <int P> hipError_t launch_fill_random(SF<P> f, int Vh, int nrhs, unsigned seed, hipStream_t s);
template <int P> hipError_t launch_check_field(SF<P> f, int Vh, int nrhs, double* out, hipStream_t s);
hipError_t launch_finish(const FinJob* j, int njob, int nblocks, int mode, hipStream_t s);
hipError_t launch_stream_copy(const void* a, void* b, long n16, hipStream_t s);  // n16 16-byte words

}  // namespace dlma
