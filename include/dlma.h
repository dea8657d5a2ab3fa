/*
 * dlma.h -- C ABI of the MI355X (gfx950) library for the hot path of distillation
 * low-mode averaging (Bushnaq et al., "Implementing noise reduction techniques
 * into the OpenQ*D package", arXiv:2201.09729).
 *
 * The method (paper Sec. 1, eq. 1-4) needs, per gauge configuration and source
 * timeslice t0:
 *   - the low modes V(t) of the spatial covariant Laplacian on every timeslice (eq. 1);
 *   - the distillation projector box(t) = V(t) V(t)^dag and its complement (eq. 1-2);
 *   - Dirac solves phi = D^-1 v for the 4N spin-diluted Laplacian modes and
 *     phi = D^-1 eta, phibar = D^-1 (1 - box(t0)) eta for the noise (eq. 3-4);
 *   - the contractions C_rest, C_mixed and C_dist (eq. 2-3).
 * D is the O(a)-improved (Wilson-clover) operator with periodic boundary
 * conditions (Sec. 2).  The paper gives no formula for it; the library uses
 *   (D psi)(x) = A(x) psi(x) - 1/2 sum_mu [(1 - g_mu) U_mu(x) psi(x+mu)
 *                                         + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu)],
 *   A(x) = (4 + m0) + csw (i/2) sum_{mu<nu} sigma_{mu nu} Fhat_{mu nu}(x),
 *   m0 = 1/(2 kappa) - 4, sigma_{mu nu} = (i/2)[g_mu, g_nu],
 *   Fhat = (Q - Q^dag)/8 from the four-leaf clover Q,
 * in the chiral basis g0 = [[0,-1],[-1,0]], gk = [[0,-i sk],[i sk,0]],
 * g5 = g0 g1 g2 g3 = diag(1,1,-1,-1).
 *
 * Conventions of every entry point:
 *   - Every function returns an int status: DLMA_OK (0) or a negative error code.
 *     dlma_last_error() returns a thread-local message for the last failure.
 *     No C++ exception crosses this boundary.
 *   - Array arguments marked "device" are caller-owned device pointers (for
 *     example a torch tensor's data_ptr()); the library never retains them after
 *     the call returns.  Arguments marked "host" are host memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  All work is
 *     enqueued on it.  Calls that return host-visible results (statistics,
 *     eigenvalues, correlators) synchronise the stream before returning.
 *   - Canonical layouts at the boundary, complex128 (re, im interleaved),
 *     x fastest, dims = {T, Z, Y, X}, direction mu: 0 = t, 1 = x, 2 = y, 3 = z:
 *       gauge   [T][Z][Y][X][mu][a][b]
 *       spinor  [nrhs][T][Z][Y][X][spin][colour]
 *       colour  [nvec][Z][Y][X][colour]  (one timeslice)
 *     All four extents must be even, >= 2 and <= 4096; the volume must be below 2^24 sites.
 *   - Internal layouts (even-odd, site-fastest structure of arrays per precision)
 *     are private to the library.
 */
#ifndef DLMA_H
#define DLMA_H

#ifdef __cplusplus
extern "C" {
#endif

#define DLMA_OK 0
#define DLMA_EINVAL (-1)      /* bad argument: dims, kappa, pointers, sizes, options */
#define DLMA_ENOMEM (-2)      /* device allocation failed */
#define DLMA_EHIP (-3)        /* HIP runtime error; message in dlma_last_error() */
#define DLMA_ENOTCONV (-4)    /* solver did not converge; outputs and statistics are written */
#define DLMA_ENAN (-5)        /* NaN or Inf in an input or produced by a solve */
#define DLMA_EUNSUPPORTED (-6)

/* Precision of a solve.  FP64: every vector and operator in double precision.
 * MIX_*: FP64 defect correction (true residual r = b - D x, norms and the
 * update x += e are FP64 on the GPU) around an inner even-odd Krylov solve whose
 * arithmetic is FP32 and whose links, clover matrices and vectors are stored in
 * FP32, FP16 (vectors with one FP32 scale per site and right-hand side) or BF16. */
#define DLMA_PREC_FP64 0
#define DLMA_PREC_MIX_FP32 1
#define DLMA_PREC_MIX_FP16 2
#define DLMA_PREC_MIX_BF16 3

typedef struct dlma_gauge_s* dlma_gauge_t;

/* Frees the device memory the library keeps cached between calls (the work buffers
 * of solves, eigensolvers and contractions, reused by later calls of the same sizes).
 * Synchronises the device.  Handles stay valid.  Returns DLMA_OK. */
int dlma_release_cache(void);

/* Library version string (static storage). */
const char* dlma_version(void);

/* Message of the last failed call on this thread (static thread-local storage). */
const char* dlma_last_error(void);

/*
 * Load a gauge configuration and build everything D needs (paper Sec. 2: O(a)
 * improved Wilson fermions; the operator above).
 *   dims   host int[4] = {T, Z, Y, X}
 *   U_dev  device, canonical gauge layout, complex128, SU(3) links (read only)
 *   kappa  hopping parameter, 0 < kappa; csw >= 0 clover coefficient
 *   out    host; receives a library-owned handle (free with dlma_free_gauge)
 * The handle holds the even-odd packed links, the clover matrices A(x) (two
 * 6x6 Hermitian chirality blocks per site), the inverse on odd sites, and
 * lower-precision copies created on first use.
 * Errors: DLMA_EINVAL (dims, kappa, csw, NULL pointer, links not unitary to
 * 1e-10, clover block not positive definite), DLMA_ENOMEM, DLMA_EHIP.
 */
int dlma_load_gauge(const int dims[4], const void* U_dev, double kappa, double csw,
                    void* stream, dlma_gauge_t* out);

/* Change kappa of a loaded configuration (re-derives A and its inverse). */
int dlma_set_mass(dlma_gauge_t g, double kappa, void* stream);

/* Release a handle and its device memory (synchronises the device). */
int dlma_free_gauge(dlma_gauge_t g);

/* Lattice extents {T, Z, Y, X} and kappa, csw of a handle. */
int dlma_gauge_info(dlma_gauge_t g, int dims_out[4], double* kappa_out, double* csw_out);

/*
 * out = D in (dagger = 0) or out = D^dag in = g5 D g5 in (dagger = 1), FP64,
 * for nrhs spinor fields in canonical layout.
 *   in, out  device, [nrhs][T][Z][Y][X][4][3] complex128; must not overlap.
 */
int dlma_apply_dw(dlma_gauge_t g, const void* in, void* out, int nrhs, int dagger, void* stream);

/*
 * The operator of the solver's inner iterations, for checking them: the
 * Schur complement of D's even-odd blocks (the even-odd reduced system that
 * dlma_solve iterates on; the paper needs D^-1 only, Sec. 2 and eq. (4)),
 *   Dhat = A_ee - D_eo A_oo^-1 D_oe   on the even sites (t + z + y + x even),
 * or Dhat^dag = g5 Dhat g5 (dagger = 1), applied by the inner stencil kernels of
 * precision prec (DLMA_PREC_*).  The even sites of `in` are rounded to the
 * storage precision (FP16: one FP32 scale per site), the links and clover
 * matrices are the storage-precision copies, A_oo^-1 D_oe in is stored at that
 * precision, and the result is rounded once more before it is widened to FP64.
 *   in, out      device, [nrhs][T][Z][Y][X][4][3] complex128; must not overlap.
 *                Odd sites of in are ignored; odd sites of out are set to 0.
 *   rhs_block    right-hand sides per thread (1 .. 4), or 0 for the launch shape
 *                the solver's autotuner picks (super_group and lds_window ignored)
 *   super_group  right-hand-side groups per super-group of the block order (0 = all)
 *   lds_window   FP16 only: 1 = stage the +-x, +-y neighbours of each block through
 *                LDS when they fit, 0 = read every neighbour from memory
 * Synchronises the stream before returning.
 * Errors: DLMA_EINVAL (handle, pointers, overlap, dagger, prec, rhs_block,
 * super_group, lds_window), DLMA_ENOMEM, DLMA_EHIP.
 */
int dlma_apply_schur(dlma_gauge_t g, const void* in, void* out, int nrhs, int dagger, int prec, int rhs_block,
                     int super_group, int lds_window, void* stream);

typedef struct {
    double tol;        /* target true relative residual |b - D x|_2 / |b|_2, FP64 (e.g. 1e-10) */
    int maxiter;       /* cap on inner CG iterations per right-hand side, all passes together */
    int max_outer;     /* cap on defect-correction passes */
    int prec;          /* DLMA_PREC_* */
    double inner_tol;  /* relative reduction of the inner residual per pass; 0 = default
                          (FP16 1e-3, BF16 1e-2, FP32 1e-5) */
    int rhs_block;     /* right-hand sides per thread in the stencil kernels: 0 = autotune, or 1 .. 4 */
    int use_x0;        /* 1: x holds the start vector on entry; 0: start from x = 0 */
    int graph_iters;   /* inner iterations captured in one hipGraph and replayed at the start of
                          each pass (replaces check_every); later convergence checks of the pass
                          follow every 2 iterations.  0 = direct launches.  Direct launches are
                          also used while dlma_profile_enable is on. */
    int check_every;   /* direct launches: inner iterations before the first host convergence
                          check of a pass (>= 1; later checks every 2); 0 = default (8) */
    int dagger;        /* 1: solve D^dag x = b (x = g5 D^-1 g5 b), the adjoint solve of a backward pass */
    int lds_window;    /* FP16 stencils stage their +-x, +-y neighbours through LDS: -1 = autotuned
                          (with rhs_block), 0 = never, 1 = when they fit */
    int inner_solver;  /* Krylov method of the inner solves on Dhat: 1 = BiCGStab on Dhat (default),
                          0 = CG on the normal equations Dhat Dhat^dag (CGNE) */
} dlma_solve_opts;

/* Fill opts with the defaults (tol 1e-10, FP64, autotuned blocks, graph_iters 8,
 * BiCGStab inner solver, ...). */
void dlma_solve_opts_default(dlma_solve_opts* opts);

typedef struct {
    int outer;         /* defect-correction passes run */
    int inner_iters;   /* inner CG iterations, all passes */
    double relres;     /* final true relative residual |b - D x| / |b|, FP64 */
    int converged;     /* 1 if relres <= tol */
} dlma_solve_stat;

typedef struct {
    const void* b;     /* device, [nrhs][T][Z][Y][X][4][3] complex128 sources */
    void* x;           /* device, same layout: solutions (start vector if use_x0) */
    int nrhs;          /* >= 0 */
} dlma_rhs_set;

/*
 * Solve D x = b for every right-hand side of every set, set i with gauge gs[i]
 * (the paper's perambulator and stochastic solves, eq. 3-4).  All sets and all
 * right-hand sides are solved together: each stencil launch covers every
 * configuration (uneven volumes allowed) and every right-hand side.
 * Algorithm: FP64 defect correction; each pass forms the Schur source
 * bhat_e = r_e - D_eo A_oo^-1 r_o, solves Dhat e = bhat_e with
 * Dhat = A_ee - D_eo A_oo^-1 D_oe in the chosen precision (BiCGStab on Dhat by
 * default, or CG on its normal equations: opts->inner_solver), and reconstructs
 * the odd sites.  After the first reconstruction the odd residual vanishes to FP64
 * rounding, so later passes compute the residual on the even sites; the odd sites
 * of the final x are checked before the solve reports convergence.  Stops per
 * right-hand side when the FP64 true relative residual is <= tol.  From x = 0 the
 * first pass skips work on timeslices where a source and its Krylov vectors are
 * exactly zero (sources on one timeslice); the results are the same as without.
 *   gs     host array of ngauge handles (1 <= ngauge <= 16)
 *   sets   host array of ngauge rhs sets
 *   stats  host array with one entry per right-hand side (sets in order), or NULL
 * Errors: DLMA_EINVAL, DLMA_ENOMEM, DLMA_EHIP, DLMA_ENAN (non-finite source or
 * iterate), DLMA_ENOTCONV (caps reached; x holds the last iterate).
 */
int dlma_solve(const dlma_gauge_t* gs, int ngauge, const dlma_rhs_set* sets,
               const dlma_solve_opts* opts, dlma_solve_stat* stats, void* stream);

typedef struct {
    double tol;        /* residual bound |lap v - lambda v| <= tol * 12 (spectrum of -lap in [0,12]) */
    int max_basis;     /* cap on the Krylov dimension (0 = default) */
    int check_every;   /* Lanczos steps between convergence checks (0 = default) */
    int cheb_degree;   /* degree of the Chebyshev filter; 0 = automatic (none for 3 L^3 < 4096), < 0 = off */
    int restart_basis; /* thick restart: basis size at which the Lanczos run keeps its best Ritz vectors
                          and continues (0 = no restarts: the basis grows to max_basis) */
    int restart_keep;  /* Ritz vectors kept per restart, nev < keep < restart_basis (0 = nev + half the rest) */
    int max_restarts;  /* cap on restarts (0 = 200) */
    int block_size;    /* > 0: block variant instead of Lanczos, a Chebyshev-filtered subspace iteration on
                          block_size vectors per timeslice, nev < block_size <= min(64, 3 L^3) */
    int block_iters;   /* cap on block iterations (0 = 200) */
} dlma_eig_opts;

/*
 * Lowest nev eigenpairs of -lap(t) for the nt timeslices t0 .. t0+nt-1 (paper
 * eq. 1, Sec. 2: the low-lying modes of the spatial covariant Laplacian on every
 * timeslice).  Lanczos with full re-orthogonalisation (two passes of classical
 * Gram-Schmidt), all timeslices advanced together.  On large timeslices the
 * Lanczos operator is a Chebyshev polynomial p(-lap) that damps the spectrum
 * above a cut estimated from a short unfiltered run and refined by a short filtered
 * one (p has the same eigenvectors; the eigenvalues returned are Rayleigh quotients
 * of lap itself, and the stopping test is the explicit residual
 * |lap v - lambda v|).  With opts->restart_basis the run is thick-restarted: the
 * basis never exceeds that many vectors, and each restart keeps the best Ritz
 * vectors and the last Lanczos vector (the projected matrix becomes arrowhead
 * plus tridiagonal).  With opts->block_size the block variant runs instead: a
 * Chebyshev-filtered subspace iteration on block_size vectors per timeslice (v0
 * is the first vector of each block, the rest seeded random), with Cholesky QR
 * and Rayleigh-Ritz steps and the same stopping test.
 *   v0       device, [nt][Z][Y][X][3] complex128 start vectors (any nonzero vectors)
 *   V_out    device, [nt][nev][Z][Y][X][3] complex128 orthonormal eigenvectors; the
 *            component of largest modulus of each vector is real and positive
 *   evals    host, [nt][nev] eigenvalues of lap(t) (<= 0), descending
 *   opts     host or NULL for defaults
 * Errors: DLMA_EINVAL, DLMA_ENOMEM, DLMA_EHIP, DLMA_ENOTCONV (basis cap reached).
 */
int dlma_lap_eigs(dlma_gauge_t g, int nev, int t0, int nt, const void* v0, void* V_out,
                  double* evals, const dlma_eig_opts* opts, void* stream);

/*
 * Distillation projector on timeslice t (paper eq. 1-2), acting on colour and
 * space and trivially on spin:
 *   mode 0: out = box(t) in;  mode 1: out = (1 - box(t)) in;  zero on every other timeslice.
 *   V_t      device, [nev][Z][Y][X][3] complex128, orthonormal columns of V(t)
 *   in, out  device, [nrhs][T][Z][Y][X][4][3] complex128 (may alias)
 */
int dlma_project(dlma_gauge_t g, int t, int nev, const void* V_t, const void* in, void* out,
                 int nrhs, int mode, void* stream);

/*
 * Allocation-free dlma_project, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid it).
 * Same arguments, same kernels and bit-identical results as dlma_project, but:
 *   - the projection coefficients live in one fixed 1 MiB device array per GPU
 *     (65536 complex doubles), held from the first call on that GPU until the
 *     process ends; right-hand sides are processed in chunks of 16384 / nev;
 *   - no device memory is allocated or freed, and no library routine that
 *     allocates is called;
 *   - the call only enqueues work on `stream` and does not synchronise it.
 * Every call on one GPU shares that array: calls on one GPU whose work can
 * overlap (different streams without ordering, or several host threads) race
 * on it and give wrong results.  Calls on one stream are ordered and safe.
 * The array keeps the last call's coefficients; no call relies on its contents.
 * Errors: DLMA_EINVAL (as dlma_project; also nev > 16384, the array's limit),
 * DLMA_EHIP (device lookup or launch failure), DLMA_EUNSUPPORTED (device index >= 64).
 */
int dlma_project_noalloc(dlma_gauge_t g, int t, int nev, const void* V_t, const void* in, void* out,
                         int nrhs, int mode, void* stream);

#define DLMA_NPARTS 7
#define DLMA_NGAMMA 2
/*
 * Correlator pieces for source timeslice t_src (paper eq. 2-4).  For
 * G in {g5 (pseudoscalar), g1/g2/g3 averaged (vector)} and X, Y in {1, P = box, Q = 1 - box}:
 *   one-end estimators  C_XY(t) = 1/N_r sum_{r,d} sum_{s,s'} (G g5)_{s s'} <phiY_{r,d,s'}, g5 G X_t phi_{r,d,s}>_t
 *   with phi^1 = phi, phi^Q = phibar, phi^P = phi - phibar (eq. 3-4), d the dilution
 *   components of one noise vector (colour and/or even-odd, each also spin-diluted),
 *   and the exact pieces
 *   C_dist = sum_{k,l} tr[g5G tau_kl Gg5 tau_kl^dag], tau = <v_k(t) x e_s, phi_{l,s'}>_t,
 *   C_QP   = sum_l sum_{s,s'} (G g5)_{s s'} <phi_{l,s'}, g5 G Q_t phi_{l,s}>_t.
 *   V_all     device, [T][nev][Z][Y][X][3]: Laplacian modes of every timeslice
 *   phi_dist  device, [4 ndist] spinors: solutions for v_l(t_src) x e_s, index l*4 + s
 *   ndist     distillation source groups passed (0 .. any): normally nev; the pieces are
 *             sums over source groups, so a caller may pass the groups in batches and
 *             add the results (C_dist and C_QP exact over the groups passed)
 *   nnoise    spin-diluted noise source groups (4 spinors each) = N_r * ndil
 *   ndil      dilution components per noise vector: 1 (spin only), 2 (even-odd),
 *             3 (colour) or 6 (colour and even-odd); must divide nnoise
 *   phi       device, [4 nnoise] spinors: D^-1 eta_{r,d,s}, index (r*ndil + d)*4 + s
 *   phibar    device, [4 nnoise] spinors: D^-1 (1 - box(t_src)) eta_{r,d,s}
 *   C_out     host, double[DLMA_NGAMMA][DLMA_NPARTS][T][2] (re, im), gamma 0 = PS, 1 = V;
 *             parts: 0 QQ_est (C_rest), 1 PQ_est (C_mixed: box at sink, 1-box at source),
 *             2 QP_est, 3 PP_est, 4 11_est (full correlator), 5 PP_exact (C_dist),
 *             6 QP_exact; time index Delta = (t - t_src) mod T.  Raw traces: no volume
 *             factor and no sign; nnoise = 0 leaves parts 0-4 zero.
 */
int dlma_correlators(dlma_gauge_t g, int t_src, int nev, const void* V_all, const void* phi_dist, int ndist,
                     int nnoise, int ndil, const void* phi, const void* phibar, double* C_out, void* stream);

/*
 * Backward of dlma_correlators (paper eq. 2-4, for gradients of correlators with
 * respect to the solutions, and through the adjoint solves to the bare mass):
 * given G = dL/dRe C + i dL/dIm C of a real loss L for every piece, with the layout
 * of C_out (host, double[DLMA_NGAMMA][DLMA_NPARTS][T][2], time index Delta), writes
 * the gradient fields such that dL = Re sum_f <grad_f, d f> to first order.  Each
 * piece c sum <A_{s'}, g5 G X_t B_s> N_{s s'} contributes
 *   grad B_s += w conj(N_{s s'}) X_t (g5 G)^dag A_{s'},  grad A_{s'} += conj(w) N_{s s'} g5 G X_t B_s
 * on timeslice t = t_src + Delta, w = G c.  All other arguments as dlma_correlators.
 *   grad_dist, grad_phi, grad_phibar  device, shaped like phi_dist, phi, phibar;
 *              overwritten on every timeslice (zero where G has no weight); must not
 *              overlap the inputs
 * Synchronises the stream.  Errors: DLMA_EINVAL (as dlma_correlators; non-finite G;
 * 2 nnoise + ndist > 65535), DLMA_ENOMEM, DLMA_EHIP.
 */
int dlma_correlators_grad(dlma_gauge_t g, int t_src, int nev, const void* V_all, const void* phi_dist, int ndist,
                          int nnoise, int ndil, const void* phi, const void* phibar, const double* G,
                          void* grad_dist, void* grad_phi, void* grad_phibar, void* stream);

/*
 * out = <a, b> = sum_i conj(a_i) b_i over n complex128 numbers (FP64, fixed
 * reduction order).  a, b device; out host double[2] (re, im).  Used by the
 * backward pass: d/dm0 of a real loss is -Re <D^-dag grad_x, x>.
 */
int dlma_dot(const void* a, const void* b, long n, double* out, void* stream);

/* ---------------------------------------------------------------- measurement */

/*
 * Kernel timing: while enabled, the stencil launches of dlma_solve and
 * dlma_bench_schur are bracketed with hipEvents on the launch stream and the
 * durations accumulated per kernel class:
 *   0 = hop_k1      odd sites, y = A_oo^-1 D_oe x                 (Dhat)
 *   1 = hop_k1_dag  odd sites, y = A_oo^-1 D_oe g5 x              (Dhat^dag)
 *   2 = hop_k2_dag  even sites, w = A_ee x - g5 D_eo y, with |w|^2  (Dhat^dag)
 *   3 = hop_k2_cg   even sites, q = A_ee w - D_eo y fused with r -= alpha q,
 *                   x += alpha w and |r|^2 (CG update, q not stored)
 *   4 = hop_k2      even sites, z = A_ee x - D_eo y               (benchmark only)
 * and the phases of dlma_lap_eigs, per Lanczos step (all timeslices of the call):
 *   5 = lap_matvec  application of -lap (or of its Chebyshev polynomial; block variant: the
 *                   filter of one iteration)
 *   6 = lap_ortho   three-term recurrence, two classical Gram-Schmidt passes, normalisation
 *                   (block variant: the two Cholesky QR passes)
 *   7 = lap_ritz    Ritz vectors and Rayleigh-quotient residual checks (block variant: the
 *                   Rayleigh-Ritz step)
 * and the stencils of the BiCGStab inner solver (K1 of both applications is class 0):
 *   8 = hop_k2_dotr even sites, v = A_ee p - D_eo y, with (rh, v)
 *   9 = hop_k2_dotx even sites, t = A_ee s - D_eo y, with (t, s) and |t|^2
 * dlma_profile_read returns the launch count, total milliseconds and total
 * algorithmic bytes (compulsory HBM traffic of the launches, summed) per class.
 */
int dlma_profile_enable(int on);
int dlma_profile_reset(void);
int dlma_profile_read(int kclass, long long* launches, double* total_ms, double* total_bytes);

/*
 * Apply the Schur operator Dhat (and Dhat^dag alternately) napply times to nrhs
 * internal random vectors in precision prec (DLMA_PREC_*: FP64, FP32, FP16, BF16
 * storage), rhs_block right-hand sides per thread (1 .. 4; 0 = autotuned).
 * Returns milliseconds per application in ms_out (host) and algorithmic bytes per
 * application in bytes_out (host).  For bandwidth measurements.
 */
int dlma_bench_schur(dlma_gauge_t g, int prec, int nrhs, int rhs_block, int napply,
                     double* ms_out, double* bytes_out, void* stream);

/*
 * Streaming copy of `bytes` (a positive multiple of 16) between two library-owned
 * device buffers, reps times (after one warm-up copy); ms_out (host) receives the
 * milliseconds per copy.  The measured peak of read + write memory bandwidth
 * (2 * bytes per copy) against which the stencil bandwidths are also quoted.
 * Synchronises the stream.  Errors: DLMA_EINVAL, DLMA_ENOMEM, DLMA_EHIP.
 */
int dlma_bench_copy(long bytes, int reps, double* ms_out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DLMA_H */
