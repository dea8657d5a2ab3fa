// Launchers of the Laplacian, Lanczos, projector and contraction kernels.
#pragma once
#include "kernels.h"

namespace dlma {

// qd (one vector per timeslice, nv = 1): also write the block partials of Re <qd, out>
// to part[t * lap_site_blocks(g) + block]
int lap_site_blocks(const Geo& g);
hipError_t launch_neg_lap(const double2* U64, const Geo& g, int t0, const double2* in, double2* out, long tsi, long tso,
                          int nt, hipStream_t s, int nv = 1, long vsi = 0, long vso = 0, const double2* qd = nullptr,
                          double* part = nullptr);
// ts*: timeslice strides of in, prev, out and qd
hipError_t launch_cheb_step(const double2* U64, const Geo& g, int t0, const double2* in, long tsi, const double2* prev, long tsp,
                            double2* out, long tso, int nt, double c1, double c2, hipStream_t s, const double2* qd = nullptr,
                            long tsqd = 0, double* part = nullptr);
hipError_t launch_rayleigh(const double2* y, const double2* ay, long n, int nvec, double* lam, double* res, hipStream_t s);
hipError_t launch_dots(const double2* a, long tsa, long isa, const double2* b, long tsb, long n, double2* out, int ostride,
                       int ni, int nt, hipStream_t s);
// Lanczos step with split reductions: alpha from the stencil's partials (nap per
// timeslice), Gram-Schmidt dots in GS_NCH element chunks, |w|^2 partials from the last
// subtraction (gs_sub_blocks(n) per timeslice) consumed by the normalisation.  prev =
// false: no beta_{j-1} q_{j-1} term (the first step after a thick restart, whose
// couplings to the kept Ritz vectors the Gram-Schmidt passes remove).
constexpr int GS_NCH = 8;
int gs_sub_blocks(long n);
hipError_t launch_lanczos_three_p(const double2* q, long tsq, long isq, double2* w, long tsw, long n, const double* apart, int nap,
                                  double* alpha, double* beta, int astride, int j, int nt, hipStream_t s, bool prev);
hipError_t launch_gs_dots(const double2* a, long tsa, long isa, const double2* b, long tsb, long n, double2* hp, int hstride, int ni,
                          int nt, hipStream_t s);
hipError_t launch_gs_sub(const double2* q, long tsq, long isq, const double2* hp, int hstride, int ni, double2* w, long tsw, long n,
                         int nt, double* npart, hipStream_t s);
hipError_t launch_scale_p(const double2* w, long tsw, double2* q, long tsq, long n, const double* npart, double* nrm, int ostride,
                          int j, int nt, hipStream_t s);
hipError_t launch_normalize_into(const double2* w, long tsw, double2* q, long tsq, long n, double* nrm, int ostride, int j, int nt,
                                 hipStream_t s);
hipError_t launch_ritz(const double2* q, long tsq, long isq, const double* S, int m, int nev, double2* y, long tsy, long n, int nt,
                       hipStream_t s);
// block eigensolver (vectors [t][k][n]; kb <= 64)
hipError_t launch_cheb_block(const double2* U64, const Geo& g, int t0, const double2* in, const double2* prev, double2* out,
                             int nt, int kb, double c1, double c2, hipStream_t s);
int block_gram_chunks(long n, int nt);
hipError_t launch_block_gram(const double2* A, const double2* B, long n, int kb, int nt, double2* part, double2* G,
                             hipStream_t s);
hipError_t launch_block_update(const double2* X, const double2* Z, long n, int kb, int kout, int nt, double2* Y, long ytstride,
                               hipStream_t s);
hipError_t launch_block_random(double2* V, long count, unsigned seed, hipStream_t s);
hipError_t launch_phase_fix(double2* y, long n, int nvec, hipStream_t s);
hipError_t launch_project(const double2* Vt, const double2* in, double2* out, const Geo& g, int t, int nev, int nrhs, int mode,
                          double2* coef, hipStream_t s);

// contractions
hipError_t launch_tproj(const double2* Vall, const double2* const* fields, int nf, const Geo& g, int nev, double2* P,
                        hipStream_t s);
// backward of the correlator contractions (see contract.hip)
struct CorrGradArgs {
    const double2* Vall;                       // [T][nev][L3][3]
    const double2 *dist, *phi, *phibar;        // input fields, canonical, fs complex numbers each
    double2 *gdist, *gphi, *gphibar;           // gradient fields (written on every timeslice)
    const double2* W1n;                        // [T][32][32]: noise groups, (phi, phibar) x spin
    const double2* W1d;                        // [T][16][16]: distillation groups, phi_dist x spin
    const double2* taun;                       // [nnoise][nact][nev][32]: WP(t) V(t)^dag F, noise groups
    const double2* taud;                       // [ndist][nact][nev][16]
    const int* tact;                           // [T]: index among the weighted timeslices, or -1
    long L3, fs;
    int nev, ndist, nnoise, nact;
};
hipError_t launch_corr_grad(const CorrGradArgs& a, int T, hipStream_t s);
hipError_t launch_spin_gram(const double2* const* A, const double2* const* B, int npair, const Geo& g, double2* G,
                            hipStream_t s);

}  // namespace dlma
