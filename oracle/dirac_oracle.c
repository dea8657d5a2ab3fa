/*
 * Plain FP64 CPU oracle for the Wilson-clover Dirac operator, its solver and the
 * spatial covariant Laplacian.  TEST INFRASTRUCTURE ONLY: it exists to check the
 * GPU library, which shares no code with it.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.
 *
 * Everything here follows the plain definitions, written for readability, not
 * speed: full-lattice operator (no even-odd splitting), explicit 4x4 gamma
 * matrices and explicit 12x12 clover matrices per site.
 *
 * Conventions (the paper fixes only "O(a)-improved Wilson fermions" and periodic
 * boundary conditions, Sec. 1 and Sec. 2):
 *   dims = {T, Z, Y, X}; site = ((t*Z + z)*Y + y)*X + x; direction mu: 0=t,1=x,2=y,3=z
 *   gauge  U[site][mu][a][b];  spinor psi[site][s][c]  (complex double)
 *   chiral basis: g0 = [[0,-1],[-1,0]], gk = [[0,-i sk],[i sk,0]], g5 = diag(1,1,-1,-1)
 *   m0 = 1/(2 kappa) - 4
 *   A(x) = (4 + m0) + csw (i/2) sum_{mu<nu} sigma_{mu nu} (x) Fhat_{mu nu}(x),
 *          sigma_{mu nu} = (i/2)[g_mu, g_nu],  Fhat = (Q - Q^dag)/8 (four-leaf clover)
 *   (D psi)(x) = A(x) psi(x) - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)
 *                                          + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ]
 *   Laplacian (paper eq. 1): (lap(t) v)(m) = -6 v(m)
 *          + sum_{j=1..3} [ U_j(m,t) v(m+j) + U_j(m-j,t)^dag v(m-j) ]
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static cplx GAM[5][4][4]; /* g0..g3, g5 */
static int gam_ready = 0;

static void init_gamma(void)
{
    if (gam_ready) return;
    memset(GAM, 0, sizeof(GAM));
    /* Pauli matrices */
    cplx sig[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
    /* g0 = [[0,-1],[-1,0]] in 2x2 blocks */
    for (int i = 0; i < 2; ++i) {
        GAM[0][i][i + 2] = -1.0;
        GAM[0][i + 2][i] = -1.0;
    }
    /* gk = [[0, -i sigma_k], [i sigma_k, 0]] */
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                GAM[k + 1][i][j + 2] = -I * sig[k][i][j];
                GAM[k + 1][i + 2][j] = I * sig[k][i][j];
            }
    /* g5 = g0 g1 g2 g3 */
    cplx t1[4][4], t2[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int k = 0; k < 4; ++k) s += GAM[0][i][k] * GAM[1][k][j];
            t1[i][j] = s;
        }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int k = 0; k < 4; ++k) s += t1[i][k] * GAM[2][k][j];
            t2[i][j] = s;
        }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int k = 0; k < 4; ++k) s += t2[i][k] * GAM[3][k][j];
            GAM[4][i][j] = s;
        }
    gam_ready = 1;
}

/* copy out the gamma matrices (for tests of the convention) */
void orc_gamma(double* out /* [5][4][4] complex */)
{
    init_gamma();
    memcpy(out, GAM, sizeof(GAM));
}

/* ---------------- lattice geometry ---------------- */

static int extent(const int* d, int mu)
{
    switch (mu) {
    case 0: return d[0]; /* t */
    case 1: return d[3]; /* x */
    case 2: return d[2]; /* y */
    default: return d[1]; /* z */
    }
}

static void coords(const int* d, long s, int c[4])
{
    int X = d[3], Y = d[2], Z = d[1];
    c[1] = (int)(s % X); s /= X;
    c[2] = (int)(s % Y); s /= Y;
    c[3] = (int)(s % Z); s /= Z;
    c[0] = (int)s;
}

static long index_of(const int* d, const int c[4])
{
    return (((long)c[0] * d[1] + c[3]) * d[2] + c[2]) * d[3] + c[1];
}

/* neighbour of site s in direction mu, step +1 or -1, periodic */
static long nbr(const int* d, long s, int mu, int step)
{
    int c[4];
    coords(d, s, c);
    int L = extent(d, mu);
    c[mu] = ((c[mu] + step) % L + L) % L;
    return index_of(d, c);
}

/* ---------------- 3x3 complex matrices ---------------- */

static const cplx* link(const cplx* U, long s, int mu) { return U + (s * 4 + mu) * 9; }

static void mm(const cplx* a, const cplx* b, cplx* c) /* c = a b */
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += a[i * 3 + k] * b[k * 3 + j];
            c[i * 3 + j] = s;
        }
}

static void dag(const cplx* a, cplx* c) /* c = a^dag */
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) c[i * 3 + j] = conj(a[j * 3 + i]);
}

static void prod4(const cplx* a, const cplx* b, const cplx* c, const cplx* e, cplx* out)
{
    cplx t1[9], t2[9];
    mm(a, b, t1);
    mm(t1, c, t2);
    mm(t2, e, out);
}

/* four-leaf clover Q_{mu nu}(x): the four plaquettes in the (mu,nu) plane that
 * touch x, each traversed counter-clockwise starting and ending at x. */
static void leaves(const int* d, const cplx* U, long x, int mu, int nu, cplx* Q)
{
    long xpm = nbr(d, x, mu, +1), xpn = nbr(d, x, nu, +1);
    long xmm = nbr(d, x, mu, -1), xmn = nbr(d, x, nu, -1);
    long xmm_pn = nbr(d, xmm, nu, +1);
    long xmm_mn = nbr(d, xmm, nu, -1);
    long xmn_pm = nbr(d, xmn, mu, +1);
    cplx A[9], B[9], C[9], E[9], L[9];
    for (int i = 0; i < 9; ++i) Q[i] = 0;

    /* U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag */
    memcpy(A, link(U, x, mu), sizeof A);
    memcpy(B, link(U, xpm, nu), sizeof B);
    dag(link(U, xpn, mu), C);
    dag(link(U, x, nu), E);
    prod4(A, B, C, E, L);
    for (int i = 0; i < 9; ++i) Q[i] += L[i];

    /* U_nu(x) U_mu(x-mu+nu)^dag U_nu(x-mu)^dag U_mu(x-mu) */
    memcpy(A, link(U, x, nu), sizeof A);
    dag(link(U, xmm_pn, mu), B);
    dag(link(U, xmm, nu), C);
    memcpy(E, link(U, xmm, mu), sizeof E);
    prod4(A, B, C, E, L);
    for (int i = 0; i < 9; ++i) Q[i] += L[i];

    /* U_mu(x-mu)^dag U_nu(x-mu-nu)^dag U_mu(x-mu-nu) U_nu(x-nu) */
    dag(link(U, xmm, mu), A);
    dag(link(U, xmm_mn, nu), B);
    memcpy(C, link(U, xmm_mn, mu), sizeof C);
    memcpy(E, link(U, xmn, nu), sizeof E);
    prod4(A, B, C, E, L);
    for (int i = 0; i < 9; ++i) Q[i] += L[i];

    /* U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^dag */
    dag(link(U, xmn, nu), A);
    memcpy(B, link(U, xmn, mu), sizeof B);
    memcpy(C, link(U, xmn_pm, nu), sizeof C);
    dag(link(U, x, mu), E);
    prod4(A, B, C, E, L);
    for (int i = 0; i < 9; ++i) Q[i] += L[i];
}

/* Fhat_{mu nu}(x) = (Q - Q^dag)/8 for the six planes mu<nu, [V][6][3][3] */
void orc_field_strength(const int* d, const cplx* U, cplx* F)
{
    long V = (long)d[0] * d[1] * d[2] * d[3];
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) {
        int p = 0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu, ++p) {
                cplx Q[9];
                leaves(d, U, x, mu, nu, Q);
                cplx* f = F + (x * 6 + p) * 9;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        f[i * 3 + j] = (Q[i * 3 + j] - conj(Q[j * 3 + i])) / 8.0;
            }
    }
}

/* A(x) as an explicit 12x12 matrix per site, index (s*3 + a), [V][12][12] */
void orc_clover(const int* d, const cplx* U, double kappa, double csw, cplx* A)
{
    init_gamma();
    long V = (long)d[0] * d[1] * d[2] * d[3];
    double m0 = 1.0 / (2.0 * kappa) - 4.0;
    cplx sigma[6][4][4];
    int p = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu, ++p)
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    cplx c = 0;
                    for (int k = 0; k < 4; ++k)
                        c += GAM[mu][i][k] * GAM[nu][k][j] - GAM[nu][i][k] * GAM[mu][k][j];
                    sigma[p][i][j] = 0.5 * I * c;
                }
    cplx* F = (cplx*)malloc(sizeof(cplx) * V * 54);
    orc_field_strength(d, U, F);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) {
        cplx* a = A + x * 144;
        for (int i = 0; i < 144; ++i) a[i] = 0;
        for (int i = 0; i < 12; ++i) a[i * 12 + i] = 4.0 + m0;
        for (int q = 0; q < 6; ++q) {
            const cplx* f = F + (x * 6 + q) * 9;
            for (int s1 = 0; s1 < 4; ++s1)
                for (int s2 = 0; s2 < 4; ++s2)
                    for (int c1 = 0; c1 < 3; ++c1)
                        for (int c2 = 0; c2 < 3; ++c2)
                            a[(s1 * 3 + c1) * 12 + s2 * 3 + c2] +=
                                csw * 0.5 * I * sigma[q][s1][s2] * f[c1 * 3 + c2];
        }
    }
    free(F);
}

/* out = D in for nrhs fields (each [V][4][3]) */
void orc_dirac(const int* d, const cplx* U, const cplx* A, const cplx* in, cplx* out, int nrhs)
{
    init_gamma();
    long V = (long)d[0] * d[1] * d[2] * d[3];
    for (int r = 0; r < nrhs; ++r) {
        const cplx* src = in + (long)r * V * 12;
        cplx* dst = out + (long)r * V * 12;
#pragma omp parallel for schedule(static)
        for (long x = 0; x < V; ++x) {
            cplx acc[12];
            const cplx* a = A + x * 144;
            const cplx* px = src + x * 12;
            for (int i = 0; i < 12; ++i) {
                cplx s = 0;
                for (int j = 0; j < 12; ++j) s += a[i * 12 + j] * px[j];
                acc[i] = s;
            }
            for (int mu = 0; mu < 4; ++mu) {
                /* forward: (1 - g_mu) U_mu(x) psi(x+mu) */
                long xf = nbr(d, x, mu, +1);
                const cplx* u = link(U, x, mu);
                const cplx* pf = src + xf * 12;
                cplx up[4][3];
                for (int s = 0; s < 4; ++s)
                    for (int a3 = 0; a3 < 3; ++a3) {
                        cplx t = 0;
                        for (int b = 0; b < 3; ++b) t += u[a3 * 3 + b] * pf[s * 3 + b];
                        up[s][a3] = t;
                    }
                for (int s = 0; s < 4; ++s)
                    for (int a3 = 0; a3 < 3; ++a3) {
                        cplx t = 0;
                        for (int s2 = 0; s2 < 4; ++s2) {
                            cplx m = (s == s2 ? 1.0 : 0.0) - GAM[mu][s][s2];
                            t += m * up[s2][a3];
                        }
                        acc[s * 3 + a3] -= 0.5 * t;
                    }
                /* backward: (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) */
                long xb = nbr(d, x, mu, -1);
                const cplx* ub = link(U, xb, mu);
                const cplx* pb = src + xb * 12;
                for (int s = 0; s < 4; ++s)
                    for (int a3 = 0; a3 < 3; ++a3) {
                        cplx t = 0;
                        for (int b = 0; b < 3; ++b) t += conj(ub[b * 3 + a3]) * pb[s * 3 + b];
                        up[s][a3] = t;
                    }
                for (int s = 0; s < 4; ++s)
                    for (int a3 = 0; a3 < 3; ++a3) {
                        cplx t = 0;
                        for (int s2 = 0; s2 < 4; ++s2) {
                            cplx m = (s == s2 ? 1.0 : 0.0) + GAM[mu][s][s2];
                            t += m * up[s2][a3];
                        }
                        acc[s * 3 + a3] -= 0.5 * t;
                    }
            }
            for (int i = 0; i < 12; ++i) dst[x * 12 + i] = acc[i];
        }
    }
}

/* out = g5 in (in place allowed) */
static void apply_g5(long V, const cplx* in, cplx* out)
{
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x)
        for (int s = 0; s < 4; ++s)
            for (int c = 0; c < 3; ++c) {
                cplx v = 0;
                for (int s2 = 0; s2 < 4; ++s2) v += GAM[4][s][s2] * in[x * 12 + s2 * 3 + c];
                out[x * 12 + s * 3 + c] = v;
            }
}

/* D^dag = g5 D g5 (gamma5-hermiticity of the Wilson-clover operator) */
void orc_dirac_dag(const int* d, const cplx* U, const cplx* A, const cplx* in, cplx* out, int nrhs)
{
    init_gamma();
    long V = (long)d[0] * d[1] * d[2] * d[3];
    cplx* t = (cplx*)malloc(sizeof(cplx) * V * 12);
    for (int r = 0; r < nrhs; ++r) {
        apply_g5(V, in + (long)r * V * 12, t);
        orc_dirac(d, U, A, t, out + (long)r * V * 12, 1);
        apply_g5(V, out + (long)r * V * 12, out + (long)r * V * 12);
    }
    free(t);
}

static double norm2(long n, const cplx* a)
{
    double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (long i = 0; i < n; ++i) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

/*
 * Solve D x = b by CG on the normal equations D^dag D x = D^dag b (CGLS form,
 * which carries s = b - D x alongside the normal-equation residual).  x holds
 * the start vector on entry.  The stopping test is on the true relative residual
 * |b - D x| / |b|, recomputed from scratch whenever the recursion claims
 * convergence; if the recursion has drifted the iteration restarts from the
 * current x.  Returns 0 if converged, 1 otherwise.
 */
int orc_cgls(const int* d, const cplx* U, const cplx* A, const cplx* b, cplx* x, double tol,
             int maxiter, int* iters_out, double* relres_out)
{
    long V = (long)d[0] * d[1] * d[2] * d[3];
    long n = V * 12;
    cplx* s = (cplx*)malloc(sizeof(cplx) * n);
    cplx* r = (cplx*)malloc(sizeof(cplx) * n);
    cplx* p = (cplx*)malloc(sizeof(cplx) * n);
    cplx* q = (cplx*)malloc(sizeof(cplx) * n);
    double bnorm = sqrt(norm2(n, b));
    int it = 0, conv = 0;
    double relres = 1.0;
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(cplx) * n);
        relres = 0.0;
        conv = 1;
        goto done;
    }
    for (;;) {
        /* (re)start: s = b - D x, r = D^dag s, p = r */
        orc_dirac(d, U, A, x, q, 1);
        for (long i = 0; i < n; ++i) s[i] = b[i] - q[i];
        relres = sqrt(norm2(n, s)) / bnorm;
        if (relres <= tol) { conv = 1; break; }
        if (it >= maxiter) break;
        orc_dirac_dag(d, U, A, s, r, 1);
        memcpy(p, r, sizeof(cplx) * n);
        double gam = norm2(n, r);
        while (it < maxiter) {
            orc_dirac(d, U, A, p, q, 1);
            double alpha = gam / norm2(n, q);
#pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) {
                x[i] += alpha * p[i];
                s[i] -= alpha * q[i];
            }
            ++it;
            if (sqrt(norm2(n, s)) / bnorm <= tol) break; /* verify at restart */
            orc_dirac_dag(d, U, A, s, r, 1);
            double gnew = norm2(n, r);
            double beta = gnew / gam;
            gam = gnew;
#pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        }
    }
done:
    if (iters_out) *iters_out = it;
    if (relres_out) *relres_out = relres;
    free(s); free(r); free(p); free(q);
    return conv ? 0 : 1;
}

/* CGLS iterations only, for timing: runs exactly `niter` iterations from x and
 * returns the recursion's relative residual |s|/|b| after them. */
double orc_cgls_fixed(const int* d, const cplx* U, const cplx* A, const cplx* b, cplx* x,
                      int niter)
{
    long V = (long)d[0] * d[1] * d[2] * d[3];
    long n = V * 12;
    cplx* s = (cplx*)malloc(sizeof(cplx) * n);
    cplx* r = (cplx*)malloc(sizeof(cplx) * n);
    cplx* p = (cplx*)malloc(sizeof(cplx) * n);
    cplx* q = (cplx*)malloc(sizeof(cplx) * n);
    double bnorm = sqrt(norm2(n, b));
    orc_dirac(d, U, A, x, q, 1);
    for (long i = 0; i < n; ++i) s[i] = b[i] - q[i];
    orc_dirac_dag(d, U, A, s, r, 1);
    memcpy(p, r, sizeof(cplx) * n);
    double gam = norm2(n, r);
    for (int it = 0; it < niter; ++it) {
        orc_dirac(d, U, A, p, q, 1);
        double alpha = gam / norm2(n, q);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            s[i] -= alpha * q[i];
        }
        orc_dirac_dag(d, U, A, s, r, 1);
        double gnew = norm2(n, r);
        double beta = gnew / gam;
        gam = gnew;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
    }
    double res = sqrt(norm2(n, s)) / bnorm;
    free(s); free(r); free(p); free(q);
    return res;
}

/* Spatial covariant Laplacian on timeslice t (paper eq. 1), acting on nvec colour
 * vectors, each [Z][Y][X][3]. */
void orc_laplacian(const int* d, const cplx* U, int t, const cplx* in, cplx* out, int nvec)
{
    long L3 = (long)d[1] * d[2] * d[3];
    for (int v = 0; v < nvec; ++v) {
        const cplx* src = in + (long)v * L3 * 3;
        cplx* dst = out + (long)v * L3 * 3;
#pragma omp parallel for schedule(static)
        for (long m = 0; m < L3; ++m) {
            long x = (long)t * L3 + m; /* 4D site index */
            cplx acc[3];
            for (int a = 0; a < 3; ++a) acc[a] = -6.0 * src[m * 3 + a];
            for (int j = 1; j <= 3; ++j) {
                long xf = nbr(d, x, j, +1), xb = nbr(d, x, j, -1);
                long mf = xf - (long)t * L3, mb = xb - (long)t * L3;
                const cplx* uf = link(U, x, j);
                const cplx* ub = link(U, xb, j);
                for (int a = 0; a < 3; ++a) {
                    cplx s = 0;
                    for (int b = 0; b < 3; ++b) {
                        s += uf[a * 3 + b] * src[mf * 3 + b];
                        s += conj(ub[b * 3 + a]) * src[mb * 3 + b];
                    }
                    acc[a] += s;
                }
            }
            for (int a = 0; a < 3; ++a) dst[m * 3 + a] = acc[a];
        }
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
