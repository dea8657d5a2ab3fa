// C ABI: Laplacian eigenmodes per timeslice (dlma_lap_eigs), the distillation
// projector (dlma_project) and the correlator pieces (dlma_correlators).
#include <algorithm>
#include <atomic>
#include <thread>
#include <cmath>
#include <complex>
#include <numeric>

#include "../../include/dlma.h"
#include "laplace.h"
#include "runtime.h"

using namespace dlma;
using cplx = std::complex<double>;

static inline hipStream_t S(void* s) { return (hipStream_t)s; }

namespace {

// Eigenvalues (and optionally eigenvectors or their last row) of the real symmetric
// tridiagonal matrix with diagonal d and off-diagonal e, by the implicit QL
// algorithm with Wilkinson-type shifts (the published method of Bowdler, Martin,
// Reinsch and Wilkinson, Numer. Math. 11 (1968) 293, the tql/imtql line of the
// Handbook for Automatic Computation and EISPACK, restated here): repeated QL sweeps
// with a shift from the trailing 2x2 block, applied as a chase of plane rotations
// from the bottom of the unreduced block upwards, with deflation when an
// off-diagonal element becomes negligible.
//   Z (m x m, row-major) receives the eigenvector matrix (columns), last its last row.
// zinit: Z holds an orthogonal matrix Q on entry and receives Q times the
// eigenvector matrix (the back-transformation of a reduction to tridiagonal form).
bool tridiag_ql(std::vector<double>& d, std::vector<double> e, std::vector<double>* Z, std::vector<double>* last,
                bool zinit = false) {
    const int n = (int)d.size();
    e.resize(n, 0.0);
    e[n - 1] = 0.0;
    if (Z && !zinit) {
        Z->assign((size_t)n * n, 0.0);
        for (int i = 0; i < n; ++i) (*Z)[(size_t)i * n + i] = 1.0;
    }
    if (last) {
        last->assign(n, 0.0);
        (*last)[n - 1] = 1.0;
    }
    const double eps = 2.220446049250313e-16;
    for (int l = 0; l < n; ++l) {
        for (int iter = 0;; ++iter) {
            int m = l;
            for (; m < n - 1; ++m) {
                double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= eps * dd) break;
            }
            if (m == l) break;
            if (iter >= 100) return false;
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = m - 1;
            bool early = false;
            for (; i >= l; --i) {
                double f = s * e[i], b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    early = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                if (Z) {
                    for (int k = 0; k < n; ++k) {
                        double* row = Z->data() + (size_t)k * n;
                        double zf = row[i + 1];
                        row[i + 1] = s * row[i] + c * zf;
                        row[i] = c * row[i] - s * zf;
                    }
                }
                if (last) {
                    double zf = (*last)[i + 1];
                    (*last)[i + 1] = s * (*last)[i] + c * zf;
                    (*last)[i] = c * (*last)[i] - s * zf;
                }
            }
            if (early) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    return true;
}

// Eigenpairs of a dense real symmetric matrix A (n x n, row-major): Householder
// reflections reduce A to tridiagonal form T = Q^T A Q, working from the last row
// upwards (the reflection of step i zeroes A[i][0..i-2] and acts on indices < i; the
// published tridiagonalisation of Martin, Reinsch and Wilkinson, Numer. Math. 11
// (1968) 181, the tred line of EISPACK, restated here),
// and the implicit QL iteration of tridiag_ql diagonalises T, its rotations applied
// to Q.  d receives the eigenvalues, Z (row-major) the eigenvectors as columns.
bool sym_eig(std::vector<double> A, int n, std::vector<double>& d, std::vector<double>& Z) {
    std::vector<double> e(n, 0.0), v(n), p(n);
    Z.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
    for (int i = n - 1; i >= 2; --i) {
        double* ai = &A[(size_t)i * n];
        double sc = 0;
        for (int k = 0; k < i; ++k) sc += ai[k] * ai[k];
        double x = std::sqrt(sc);
        if (x == 0.0) { e[i - 1] = 0.0; continue; }
        // reflection H = 1 - v v^T / h on indices 0..i-1 mapping row i's part onto e_{i-1}
        const double alpha = ai[i - 1] > 0 ? -x : x;
        for (int k = 0; k < i; ++k) v[k] = ai[k];
        v[i - 1] -= alpha;
        double h = 0;
        for (int k = 0; k < i; ++k) h += v[k] * v[k];
        h *= 0.5;
        if (h == 0.0) { e[i - 1] = ai[i - 1]; continue; }
        // A' = H A H on the leading i x i block: p = A v / h, K = v.p / (2h), q = p - K v, A' = A - v q^T - q v^T
        double K = 0;
        for (int r = 0; r < i; ++r) {
            const double* ar = &A[(size_t)r * n];
            double acc = 0;
            for (int c = 0; c < i; ++c) acc += ar[c] * v[c];
            p[r] = acc / h;
            K += v[r] * p[r];
        }
        K /= 2.0 * h;
        for (int r = 0; r < i; ++r) p[r] -= K * v[r];
        for (int r = 0; r < i; ++r) {
            double* ar = &A[(size_t)r * n];
            for (int c = 0; c < i; ++c) ar[c] -= v[r] * p[c] + p[r] * v[c];
        }
        for (int k = 0; k < i - 1; ++k) { ai[k] = 0.0; A[(size_t)k * n + i] = 0.0; }
        ai[i - 1] = alpha;
        A[(size_t)(i - 1) * n + i] = alpha;
        e[i - 1] = alpha;
        // Q = Q H (columns 0..i-1)
        for (int r = 0; r < n; ++r) {
            double* zr = &Z[(size_t)r * n];
            double acc = 0;
            for (int k = 0; k < i; ++k) acc += zr[k] * v[k];
            acc /= h;
            if (acc != 0.0)
                for (int k = 0; k < i; ++k) zr[k] -= acc * v[k];
        }
    }
    if (n >= 2) e[0] = A[1];
    d.resize(n);
    for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
    e.resize(n - 1 > 0 ? n - 1 : 0);
    return tridiag_ql(d, e, &Z, nullptr, true);
}

// Eigenpairs of a complex Hermitian n x n matrix A (row-major): Householder
// reflections I - 2 v v^H reduce A to Hermitian tridiagonal form (column k below the
// diagonal mapped onto a multiple of e_{k+1}); a diagonal of unit phases makes the
// off-diagonals real and non-negative; tridiag_ql diagonalises the real tridiagonal
// matrix; the eigenvectors are Q D Y.  d: eigenvalues (unsorted), Z: eigenvectors
// as columns (row-major).
bool herm_eig(std::vector<cplx> A, int n, std::vector<double>& d, std::vector<cplx>& Z) {
    std::vector<cplx> Q((size_t)n * n, 0.0), v(n), p(n), q(n);
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
    auto a = [&](int r, int c) -> cplx& { return A[(size_t)r * n + c]; };
    for (int k = 0; k + 2 < n; ++k) {
        double xn2 = 0;
        for (int i = k + 1; i < n; ++i) xn2 += std::norm(a(i, k));
        const double xn = std::sqrt(xn2);
        if (xn == 0.0) continue;
        const cplx x0 = a(k + 1, k);
        const cplx ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cplx(1.0, 0.0);
        const cplx alpha = -ph * xn;
        double vn2 = 0;
        for (int i = k + 1; i < n; ++i) v[i] = a(i, k);
        v[k + 1] -= alpha;
        for (int i = k + 1; i < n; ++i) vn2 += std::norm(v[i]);
        if (vn2 == 0.0) continue;
        const double vn = std::sqrt(vn2);
        for (int i = k + 1; i < n; ++i) v[i] /= vn;
        // trailing block: A' = A - 2 v q^H - 2 q v^H with p = A v, q = p - (v^H p) v
        cplx vp = 0;
        for (int r = k + 1; r < n; ++r) {
            cplx acc = 0;
            for (int c = k + 1; c < n; ++c) acc += a(r, c) * v[c];
            p[r] = acc;
            vp += std::conj(v[r]) * acc;
        }
        for (int r = k + 1; r < n; ++r) q[r] = p[r] - vp * v[r];
        for (int r = k + 1; r < n; ++r)
            for (int c = k + 1; c < n; ++c) a(r, c) -= 2.0 * (v[r] * std::conj(q[c]) + q[r] * std::conj(v[c]));
        a(k + 1, k) = alpha;
        a(k, k + 1) = std::conj(alpha);
        for (int i = k + 2; i < n; ++i) a(i, k) = a(k, i) = 0.0;
        // Q = Q H
        for (int r = 0; r < n; ++r) {
            cplx acc = 0;
            for (int c = k + 1; c < n; ++c) acc += Q[(size_t)r * n + c] * v[c];
            for (int c = k + 1; c < n; ++c) Q[(size_t)r * n + c] -= 2.0 * acc * std::conj(v[c]);
        }
    }
    d.resize(n);
    std::vector<double> e(n > 1 ? n - 1 : 0);
    std::vector<cplx> delta(n, 1.0);
    for (int i = 0; i < n; ++i) d[i] = a(i, i).real();
    for (int i = 0; i + 1 < n; ++i) {
        const cplx ei = a(i + 1, i);
        const double ae = std::abs(ei);
        e[i] = ae;
        delta[i + 1] = ae > 0 ? delta[i] * ei / ae : delta[i];
    }
    std::vector<double> Y;
    if (!tridiag_ql(d, e, &Y, nullptr)) return false;
    Z.assign((size_t)n * n, 0.0);
    for (int r = 0; r < n; ++r)
        for (int i = 0; i < n; ++i) {
            const cplx qd = Q[(size_t)r * n + i] * delta[i];
            if (qd == cplx(0.0, 0.0)) continue;
            for (int j = 0; j < n; ++j) Z[(size_t)r * n + j] += qd * Y[(size_t)i * n + j];
        }
    return true;
}

// Z = D R^-1 for the Cholesky factor R (upper, G' = R^H R) of G' = D G D, D =
// diag(G_ii^-1/2): X Z has orthonormal columns when G = X^H X.  False if G' is not
// numerically positive definite.
bool chol_orth_factor(const std::vector<cplx>& G, int n, std::vector<cplx>& Z) {
    std::vector<double> dg(n);
    for (int i = 0; i < n; ++i) {
        const double gii = G[(size_t)i * n + i].real();
        if (!(gii > 0)) return false;
        dg[i] = 1.0 / std::sqrt(gii);
    }
    std::vector<cplx> R((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double s = G[(size_t)j * n + j].real() * dg[j] * dg[j];
        for (int k = 0; k < j; ++k) s -= std::norm(R[(size_t)k * n + j]);
        if (!(s > 0)) return false;
        const double rjj = std::sqrt(s);
        R[(size_t)j * n + j] = rjj;
        for (int i = j + 1; i < n; ++i) {
            cplx t = G[(size_t)j * n + i] * dg[j] * dg[i];
            for (int k = 0; k < j; ++k) t -= std::conj(R[(size_t)k * n + j]) * R[(size_t)k * n + i];
            R[(size_t)j * n + i] = t / rjj;
        }
    }
    // R^-1 by back substitution, column by column; then the row scaling by D
    Z.assign((size_t)n * n, 0.0);
    for (int c = 0; c < n; ++c) {
        Z[(size_t)c * n + c] = 1.0 / R[(size_t)c * n + c];
        for (int i = c - 1; i >= 0; --i) {
            cplx acc = 0;
            for (int k = i + 1; k <= c; ++k) acc += R[(size_t)i * n + k] * Z[(size_t)k * n + c];
            Z[(size_t)i * n + c] = -acc / R[(size_t)i * n + i];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < n; ++c) Z[(size_t)i * n + c] *= dg[i];
    return true;
}

std::vector<int> argsort(const std::vector<double>& v) {
    std::vector<int> idx(v.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return v[a] < v[b]; });
    return idx;
}

// f(t) for t = 0 .. n-1 on the host's cores (the per-timeslice tridiagonal problems
// are independent); false if any call returned false
template <class F> bool parallel_for(int n, F f) {
    const int nth = std::max(1, std::min<int>(n, (int)std::thread::hardware_concurrency()));
    std::atomic<int> next(0);
    std::atomic<bool> all(true);
    auto work = [&]() {
        for (int t; (t = next.fetch_add(1)) < n;)
            if (!f(t)) all = false;
    };
    std::vector<std::thread> th;
    for (int i = 1; i < nth; ++i) th.emplace_back(work);
    work();
    for (auto& x : th) x.join();
    return all;
}

}  // namespace

// Block variant: Chebyshev-filtered subspace iteration on a block of kb > nev vectors
// per timeslice.  Each iteration filters the block with T_deg((c - (-lap))/e), which
// damps [cut, 12] (cut = the block's largest Ritz value), orthonormalises it (Cholesky
// QR, twice, after scaling the columns to unit length), and takes the Rayleigh-Ritz
// vectors of the block.  The degree is the largest (at most 60) with
// T_deg at the lowest Ritz value below 1e8, so the filtered columns keep a dynamic
// range the Cholesky QR resolves.  Stops when the nev lowest Ritz pairs have
// |lap v - lambda v| <= tol * 12.  All timeslices advance together; the block
// operations (filter, Gram matrices, basis updates) are batched over the block.
static int block_eigs(Gauge* g, int nev, int t0, int nt, const double2* v0, double2* Vo, double* evals, double tol,
                      const dlma_eig_opts* opts, hipStream_t s) {
    const long L3 = (long)g->dims[1] * g->dims[2] * g->dims[3];
    const long n = 3 * L3;
    const int kb = opts->block_size;
    if (kb <= nev || kb > 64 || kb > n) return fail(DLMA_EINVAL, "block_size must satisfy nev < block_size <= min(64, 3 L^3)");
    const int maxit = opts->block_iters > 0 ? opts->block_iters : 200;
    const size_t bsz = (size_t)nt * kb * n;
    Buf pool[4], Part, Gd, Zd, LR;
    for (auto& b : pool) DLMA_TRY(b.allocate(sizeof(double2) * bsz));
    const int nc = block_gram_chunks(n, nt);
    DLMA_TRY(Part.allocate(sizeof(double2) * (size_t)nt * nc * kb * kb));
    DLMA_TRY(Gd.allocate(sizeof(double2) * (size_t)nt * kb * kb));
    DLMA_TRY(Zd.allocate(sizeof(double2) * (size_t)nt * kb * kb));
    DLMA_TRY(LR.allocate(sizeof(double) * 2 * (size_t)nt * kb));
    double2* buf[4] = {pool[0].as<double2>(), pool[1].as<double2>(), pool[2].as<double2>(), pool[3].as<double2>()};
    int iX = 0, iW = 1;  // current block and -lap of it; the other two are free
    auto free_pair = [&](int& a, int& b) {
        int f[2], k = 0;
        for (int i = 0; i < 4 && k < 2; ++i)
            if (i != iX && i != iW) f[k++] = i;
        a = f[0];
        b = f[1];
    };
    const double2* U64 = g->U64.as<double2>();
    Profiler& prof = Profiler::get();
    const double vec_b = 16.0 * n * nt * kb, link_b = 3.0 * 2.0 * 9.0 * 16.0 * L3 * nt;
    std::vector<cplx> hG((size_t)nt * kb * kb), hZ((size_t)nt * kb * kb);
    std::vector<double> lam((size_t)nt * kb), res((size_t)nt * kb);
    auto gram = [&](const double2* A, const double2* B) -> int {
        DLMA_HIP(launch_block_gram(A, B, n, kb, nt, Part.as<double2>(), Gd.as<double2>(), s));
        DLMA_HIP(hipMemcpyAsync(hG.data(), Gd.p, sizeof(double2) * hG.size(), hipMemcpyDeviceToHost, s));
        DLMA_HIP(hipStreamSynchronize(s));
        return DLMA_OK;
    };
    auto orth = [&]() -> int {  // Cholesky QR twice on the current block
        hipEvent_t ev = nullptr;
        if (prof.on) prof.begin(0, 0.0, s, ev);
        for (int pass = 0; pass < 2; ++pass) {
            DLMA_TRY(gram(buf[iX], buf[iX]));
            for (int t = 0; t < nt; ++t) {
                std::vector<cplx> Gt(hG.begin() + (size_t)t * kb * kb, hG.begin() + (size_t)(t + 1) * kb * kb), Zt;
                if (!chol_orth_factor(Gt, kb, Zt)) return fail(DLMA_ENOTCONV, "block eigensolver: the filtered block lost rank");
                std::copy(Zt.begin(), Zt.end(), hZ.begin() + (size_t)t * kb * kb);
            }
            int f0, f1;
            free_pair(f0, f1);
            DLMA_HIP(hipMemcpyAsync(Zd.p, hZ.data(), sizeof(double2) * hZ.size(), hipMemcpyHostToDevice, s));
            DLMA_HIP(launch_block_update(buf[iX], Zd.as<double2>(), n, kb, kb, nt, buf[f0], (long)kb * n, s));
            iX = f0;
        }
        DLMA_HIP(hipStreamSynchronize(s));  // hZ is rewritten next
        if (prof.on) prof.end(ev, KC_LAP_ORTHO, 2.0 * (2.0 * vec_b + 2.0 * vec_b), s);
        return DLMA_OK;
    };
    auto rayleigh_ritz = [&]() -> int {  // Ritz vectors of the (orthonormal) block, ascending
        hipEvent_t ev = nullptr;
        if (prof.on) prof.begin(0, 0.0, s, ev);
        DLMA_HIP(launch_neg_lap(U64, g->geo, t0, buf[iX], buf[iW], (long)kb * n, (long)kb * n, nt, s, kb, n, n));
        DLMA_TRY(gram(buf[iX], buf[iW]));
        for (int t = 0; t < nt; ++t) {
            std::vector<cplx> Ht(hG.begin() + (size_t)t * kb * kb, hG.begin() + (size_t)(t + 1) * kb * kb), Zc;
            for (int i = 0; i < kb; ++i)  // symmetrise the rounding
                for (int j = 0; j < i; ++j) {
                    const cplx a = 0.5 * (Ht[(size_t)i * kb + j] + std::conj(Ht[(size_t)j * kb + i]));
                    Ht[(size_t)i * kb + j] = a;
                    Ht[(size_t)j * kb + i] = std::conj(a);
                }
            for (int i = 0; i < kb; ++i) Ht[(size_t)i * kb + i] = Ht[(size_t)i * kb + i].real();
            std::vector<double> d;
            if (!herm_eig(Ht, kb, d, Zc)) return fail(DLMA_EHIP, "block eigensolver: projected eigenproblem did not converge");
            std::vector<int> idx = argsort(d);
            for (int j = 0; j < kb; ++j)
                for (int i = 0; i < kb; ++i) hZ[(size_t)t * kb * kb + (size_t)i * kb + j] = Zc[(size_t)i * kb + idx[j]];
        }
        int f0, f1;
        free_pair(f0, f1);
        DLMA_HIP(hipMemcpyAsync(Zd.p, hZ.data(), sizeof(double2) * hZ.size(), hipMemcpyHostToDevice, s));
        DLMA_HIP(launch_block_update(buf[iX], Zd.as<double2>(), n, kb, kb, nt, buf[f0], (long)kb * n, s));
        DLMA_HIP(launch_block_update(buf[iW], Zd.as<double2>(), n, kb, kb, nt, buf[f1], (long)kb * n, s));
        iX = f0;
        iW = f1;
        double* dl = LR.as<double>();
        DLMA_HIP(launch_rayleigh(buf[iX], buf[iW], n, nt * kb, dl, dl + (size_t)nt * kb, s));
        DLMA_HIP(hipMemcpyAsync(lam.data(), dl, sizeof(double) * lam.size(), hipMemcpyDeviceToHost, s));
        DLMA_HIP(hipMemcpyAsync(res.data(), dl + (size_t)nt * kb, sizeof(double) * res.size(), hipMemcpyDeviceToHost, s));
        DLMA_HIP(hipStreamSynchronize(s));
        if (prof.on) prof.end(ev, KC_LAP_RITZ, link_b + 8.0 * vec_b, s);
        return DLMA_OK;
    };
    // start: seeded random block whose first column is the caller's start vector
    DLMA_HIP(launch_block_random(buf[iX], (long)bsz, 0x5eedu + (unsigned)t0, s));
    DLMA_HIP(hipMemcpy2DAsync(buf[iX], sizeof(double2) * kb * n, v0, sizeof(double2) * n, sizeof(double2) * n, nt,
                              hipMemcpyDeviceToDevice, s));
    DLMA_TRY(orth());
    DLMA_TRY(rayleigh_ritz());
    bool conv = false;
    for (int it = 0;; ++it) {
        conv = true;
        for (int t = 0; t < nt && conv; ++t)
            for (int k = 0; k < nev; ++k)
                if (!(res[(size_t)t * kb + k] <= tol * 12.0)) { conv = false; break; }
        if (conv || it >= maxit) break;
        double cut = 0, lo = 12.0;
        for (int t = 0; t < nt; ++t) {
            cut = std::max(cut, lam[(size_t)t * kb + kb - 1]);
            lo = std::min(lo, lam[(size_t)t * kb]);
        }
        cut = std::min(cut, 11.5);
        const double cc = 0.5 * (cut + 12.0), ee = 0.5 * (12.0 - cut);
        const double x1 = std::max((cc - lo) / ee, 1.0 + 1e-12);
        int deg = 4;
        while (deg < 60 && std::cosh((deg + 1) * std::acosh(x1)) < 1e8) ++deg;
        hipEvent_t ev = nullptr;
        if (prof.on) prof.begin(0, 0.0, s, ev);
        int f0, f1;
        free_pair(f0, f1);
        int ia = iX, ib = f0, ic = f1;  // the recurrence rotates through X, the free pair and W
        DLMA_HIP(launch_cheb_block(U64, g->geo, t0, buf[ia], nullptr, buf[ib], nt, kb, cc, 1.0 / ee, s));
        for (int k = 2; k <= deg; ++k) {
            DLMA_HIP(launch_cheb_block(U64, g->geo, t0, buf[ib], buf[ia], buf[ic], nt, kb, cc, 2.0 / ee, s));
            const int t = ia;
            ia = ib;
            ib = ic;
            ic = (k == 2) ? iW : t;  // W is free until the next Rayleigh-Ritz step
        }
        if (prof.on) prof.end(ev, KC_LAP_MATVEC, deg * (link_b + 3.0 * vec_b), s);
        // the filtered block is in ib; W takes any buffer other than it
        iX = ib;
        iW = (ia != iX) ? ia : ic;
        DLMA_TRY(orth());
        DLMA_TRY(rayleigh_ritz());
    }
    // the nev lowest Ritz pairs, ascending in -lap (descending in lap)
    DLMA_HIP(hipMemcpy2DAsync(Vo, sizeof(double2) * nev * n, buf[iX], sizeof(double2) * kb * n, sizeof(double2) * nev * n, nt,
                              hipMemcpyDeviceToDevice, s));
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k < nev; ++k) evals[(size_t)t * nev + k] = -lam[(size_t)t * kb + k];
    DLMA_HIP(launch_phase_fix(Vo, n, nev * nt, s));
    DLMA_HIP(hipStreamSynchronize(s));
    if (prof.on) prof.collect();
    if (!conv) return fail(DLMA_ENOTCONV, "block eigensolver did not reach the tolerance within block_iters iterations");
    return DLMA_OK;
}

extern "C" int dlma_lap_eigs(dlma_gauge_t h, int nev, int t0, int nt, const void* v0, void* V_out, double* evals,
                             const dlma_eig_opts* opts, void* stream) {
    Gauge* g = (Gauge*)h;
    if (!g) return fail(DLMA_EINVAL, "NULL handle");
    if (!v0 || !V_out || !evals) return fail(DLMA_EINVAL, "NULL pointer");
    const int T = g->dims[0];
    const long L3 = (long)g->dims[1] * g->dims[2] * g->dims[3];
    const long n = 3 * L3;
    if (nt < 1 || t0 < 0 || t0 + nt > T) return fail(DLMA_EINVAL, "timeslices t0..t0+nt-1 must lie in [0, T)");
    if (nev < 1 || nev > n) return fail(DLMA_EINVAL, "nev must be in [1, 3 L^3]");
    const double tol = (opts && opts->tol > 0) ? opts->tol : 1e-10;
    if (opts && opts->block_size > 0) return block_eigs(g, nev, t0, nt, (const double2*)v0, (double2*)V_out, evals, tol, opts, S(stream));
    // thick restart: the basis holds at most restart_basis vectors; at that size the
    // run keeps `keep` Ritz vectors of the wanted end and the last Lanczos vector
    const bool restart = opts && opts->restart_basis > 0;
    int maxm = restart ? opts->restart_basis
                       : ((opts && opts->max_basis > 0) ? opts->max_basis : (int)std::min<long>(n, 20L * nev + 200));
    maxm = (int)std::min<long>(maxm, n);
    if (maxm < nev) return fail(DLMA_EINVAL, "max_basis must be >= nev");
    int keep = 0, max_restarts = 0;
    if (restart) {
        keep = opts->restart_keep > 0 ? opts->restart_keep : nev + (maxm - nev) / 2;
        max_restarts = opts->max_restarts > 0 ? opts->max_restarts : 200;
        if (!(keep > nev && keep < maxm - 1)) return fail(DLMA_EINVAL, "need nev < restart_keep < restart_basis - 1");
    }
    const int check = (opts && opts->check_every > 0) ? opts->check_every : 10;
    int deg = opts ? opts->cheb_degree : 0;
    if (deg == 0) deg = n >= 4096 ? 24 : 0;
    if (deg < 0) deg = 0;
    hipStream_t s = S(stream);
    const long isq = n, tsq = (long)(maxm + 1) * n;
    Buf Q, R[3], Hc, AB, AY, LR, RZ, PA, PN;
    DLMA_TRY(Q.allocate(sizeof(double2) * tsq * nt));
    for (auto& b : R) DLMA_TRY(b.allocate(sizeof(double2) * n * nt));
    DLMA_TRY(Hc.allocate(sizeof(double2) * (size_t)(maxm + 1) * nt * GS_NCH));
    // block partials of alpha (from the stencil) and of |w|^2 (from the last Gram-Schmidt pass)
    DLMA_TRY(PA.allocate(sizeof(double) * (size_t)lap_site_blocks(g->geo) * nt));
    DLMA_TRY(PN.allocate(sizeof(double) * (size_t)gs_sub_blocks(n) * nt));
    DLMA_TRY(AB.allocate(sizeof(double) * 2 * (size_t)maxm * nt + 64));
    DLMA_TRY(AY.allocate(sizeof(double2) * (size_t)nt * nev * n));
    DLMA_TRY(LR.allocate(sizeof(double) * 2 * (size_t)nt * nev));
    if (restart) DLMA_TRY(RZ.allocate(sizeof(double2) * (size_t)nt * keep * n));
    double2* q = Q.as<double2>();
    double* alpha = AB.as<double>();
    double* beta = alpha + (size_t)maxm * nt;
    double* dlam = LR.as<double>();
    double* dres = dlam + (size_t)nt * nev;
    double2* Vo = (double2*)V_out;
    const double2* U64 = g->U64.as<double2>();
    std::vector<double> ha((size_t)maxm * nt), hb((size_t)maxm * nt), hlam((size_t)nt * nev), hres((size_t)nt * nev);
    // after a thick restart: kept Ritz values theta and their couplings sigma to the
    // basis vector at position karrow (the Lanczos vector carried over)
    int karrow = 0;
    std::vector<double> theta, sigma;
    int cur_deg = 0;
    double cc = 0, ee = 1;
    // phase timing for the profiler (events bracket each phase on the stream);
    // bytes: the algorithmic traffic of the phase (matvec: links of the timeslice
    // plus the input and output vectors; Gram-Schmidt: every basis vector read twice
    // per pass plus w read and written)
    Profiler& prof = Profiler::get();
    auto t_begin = [&](hipEvent_t& e) {
        if (prof.on) prof.begin(0, 0.0, s, e);
    };
    auto t_end = [&](hipEvent_t e, int kc, double bytes) {
        if (prof.on) prof.end(e, kc, bytes, s);
    };
    const double vec_b = 16.0 * n * nt, link_b = 3.0 * 2.0 * 9.0 * 16.0 * L3 * nt;

    // w = B q_j with B = -lap (cur_deg = 0) or T_deg((c - (-lap))/e); the last stencil
    // also writes the block partials of Re <q_j, w> (alpha_j) to PA.  The recurrence
    // reads q_j in place (stride tsq) and rotates through R[0..2].
    double* apart = PA.as<double>();
    const int nap = lap_site_blocks(g->geo);
    auto apply_op = [&](const double2* qj, double2*& w) -> int {
        if (cur_deg == 0) {
            DLMA_HIP(launch_neg_lap(U64, g->geo, t0, qj, R[0].as<double2>(), tsq, n, nt, s, 1, 0, 0, qj, apart));
            w = R[0].as<double2>();
            return DLMA_OK;
        }
        const double2* a = qj;
        long tsa = tsq;
        double2 *b = R[1].as<double2>(), *c = R[2].as<double2>(), *spare = R[0].as<double2>();
        const bool last1 = cur_deg == 1;
        DLMA_HIP(launch_cheb_step(U64, g->geo, t0, a, tsa, nullptr, 0, b, n, nt, cc, 1.0 / ee, s, last1 ? qj : nullptr, tsq,
                                  last1 ? apart : nullptr));
        for (int k = 2; k <= cur_deg; ++k) {
            const bool last = k == cur_deg;
            DLMA_HIP(launch_cheb_step(U64, g->geo, t0, b, n, a, tsa, c, n, nt, cc, 2.0 / ee, s, last ? qj : nullptr, tsq,
                                      last ? apart : nullptr));
            double2* freed = (a == qj) ? spare : const_cast<double2*>(a);  // never write q_j
            a = b;
            tsa = n;
            b = c;
            c = freed;
        }
        w = b;
        return DLMA_OK;
    };
    // Eigenpairs of timeslice t's m-column projected matrix: the Lanczos tridiagonal
    // (alpha, beta) until the first thick restart; after it the kept Ritz values on the
    // diagonal, coupled to column karrow by sigma, then the tridiagonal continuation.
    // ha, hb hold alpha, beta (copied from the device by the caller).
    auto proj_eig = [&](int t, int m, std::vector<double>& d, std::vector<double>* Z, std::vector<double>* last) -> bool {
        const double* at = ha.data() + (size_t)t * maxm;
        const double* bt = hb.data() + (size_t)t * maxm;
        if (karrow == 0) {
            d.assign(at, at + m);
            std::vector<double> e(bt, bt + std::max(0, m - 1));
            return tridiag_ql(d, e, Z, last);
        }
        std::vector<double> A((size_t)m * m, 0.0), Zl;
        for (int i = 0; i < karrow; ++i) {
            A[(size_t)i * m + i] = theta[(size_t)t * keep + i];
            A[(size_t)i * m + karrow] = A[(size_t)karrow * m + i] = sigma[(size_t)t * keep + i];
        }
        for (int j = karrow; j < m; ++j) {
            A[(size_t)j * m + j] = at[j];
            if (j + 1 < m) A[(size_t)j * m + j + 1] = A[(size_t)(j + 1) * m + j] = bt[j];
        }
        if (!sym_eig(std::move(A), m, d, Zl)) return false;
        if (last) last->assign(Zl.begin() + (size_t)(m - 1) * m, Zl.begin() + (size_t)m * m);
        if (Z) *Z = std::move(Zl);
        return true;
    };
    // Ritz vectors of the m-column projected matrices (the nev smallest or largest Ritz
    // values) into V_out, then their Rayleigh quotients and residuals for -lap
    auto ritz_check = [&](int m, bool largest, bool& ok) -> int {
        DLMA_HIP(hipMemcpyAsync(ha.data(), alpha, sizeof(double) * maxm * nt, hipMemcpyDeviceToHost, s));
        DLMA_HIP(hipMemcpyAsync(hb.data(), beta, sizeof(double) * maxm * nt, hipMemcpyDeviceToHost, s));
        DLMA_HIP(hipStreamSynchronize(s));
        std::vector<double> Sall((size_t)nt * m * nev);
        const bool solved = parallel_for(nt, [&](int t) {
            std::vector<double> d, Z;
            if (!proj_eig(t, m, d, &Z, nullptr)) return false;
            std::vector<int> idx = argsort(d);
            if (largest) std::reverse(idx.begin(), idx.end());
            for (int k = 0; k < nev; ++k)
                for (int i = 0; i < m; ++i) Sall[((size_t)t * m + i) * nev + k] = Z[(size_t)i * m + idx[k]];
            return true;
        });
        if (!solved) return fail(DLMA_EHIP, "tridiagonal eigensolver did not converge");
        Buf Sd;
        DLMA_TRY(Sd.allocate(sizeof(double) * Sall.size()));
        DLMA_HIP(hipMemcpyAsync(Sd.p, Sall.data(), sizeof(double) * Sall.size(), hipMemcpyHostToDevice, s));
        hipEvent_t ev = nullptr;
        t_begin(ev);
        DLMA_HIP(launch_ritz(q, tsq, isq, Sd.as<double>(), m, nev, Vo, (long)nev * n, n, nt, s));
        DLMA_HIP(launch_neg_lap(U64, g->geo, t0, Vo, AY.as<double2>(), (long)nev * n, (long)nev * n, nt, s, nev, n, n));
        DLMA_HIP(launch_rayleigh(Vo, AY.as<double2>(), n, nt * nev, dlam, dres, s));
        t_end(ev, KC_LAP_RITZ, (double)m * vec_b + nev * (link_b + 4.0 * vec_b));
        DLMA_HIP(hipMemcpyAsync(hlam.data(), dlam, sizeof(double) * nt * nev, hipMemcpyDeviceToHost, s));
        DLMA_HIP(hipMemcpyAsync(hres.data(), dres, sizeof(double) * nt * nev, hipMemcpyDeviceToHost, s));
        DLMA_HIP(hipStreamSynchronize(s));
        if (prof.on) prof.collect();
        ok = true;
        for (double r : hres)
            if (!(r <= tol * 12.0)) ok = false;
        return DLMA_OK;
    };
    // Up to msteps Lanczos steps with the current operator from q_0 = v0/|v0|.  With
    // thick restart the basis never exceeds maxm vectors: when it is full, the keep
    // Ritz vectors of the wanted end replace it, the last Lanczos vector follows them,
    // and the run continues from there (convergence is tested once per cycle).
    auto lanczos = [&](long msteps, bool largest, bool checks, int& m, bool& conv, const double2* start) -> int {
        conv = false;
        m = 0;
        karrow = 0;
        int next_check = check, restarts = 0;
        DLMA_HIP(launch_normalize_into(start, n, q, tsq, n, beta, maxm, 0, nt, s));
        DLMA_HIP(hipMemcpyAsync(hb.data(), beta, sizeof(double) * maxm * nt, hipMemcpyDeviceToHost, s));
        DLMA_HIP(hipStreamSynchronize(s));
        for (int t = 0; t < nt; ++t)
            if (!(hb[(size_t)t * maxm] > 0) || !std::isfinite(hb[(size_t)t * maxm]))
                return fail(DLMA_EINVAL, "start vector is zero or not finite");
        int j = 0;  // position of the vector the next step expands
        for (long step = 0; step < msteps; ++step) {
            double2* w = nullptr;
            hipEvent_t ev = nullptr;
            t_begin(ev);
            DLMA_TRY(apply_op(q + (long)j * isq, w));
            t_end(ev, KC_LAP_MATVEC, (cur_deg > 0 ? cur_deg : 1) * (link_b + 2.0 * vec_b));
            t_begin(ev);
            DLMA_HIP(launch_lanczos_three_p(q, tsq, isq, w, n, n, apart, nap, alpha, beta, maxm, j, nt, s, j > karrow));
            for (int pass = 0; pass < 2; ++pass) {  // classical Gram-Schmidt against all q_i, twice
                DLMA_HIP(launch_gs_dots(q, tsq, isq, w, n, n, Hc.as<double2>(), maxm + 1, j + 1, nt, s));
                DLMA_HIP(launch_gs_sub(q, tsq, isq, Hc.as<double2>(), maxm + 1, j + 1, w, n, n, nt,
                                       pass == 1 ? PN.as<double>() : nullptr, s));
            }
            DLMA_HIP(launch_scale_p(w, n, q + (long)(j + 1) * isq, tsq, n, PN.as<double>(), beta, maxm, j, nt, s));
            t_end(ev, KC_LAP_ORTHO, (4.0 * (j + 1) + 8.0) * vec_b);
            m = ++j;
            const bool last_step = step + 1 == msteps;
            if (!checks) continue;
            if (restart) {
                if (m < maxm && !last_step) continue;
            } else {
                // convergence checks every `check` steps, spaced out to m/16 on long runs
                // (each one solves the m x m tridiagonal problems on the host)
                if (m < nev || (m < next_check && !last_step)) continue;
                next_check = m + std::max(check, m / 16);
            }
            DLMA_HIP(hipMemcpyAsync(ha.data(), alpha, sizeof(double) * maxm * nt, hipMemcpyDeviceToHost, s));
            DLMA_HIP(hipMemcpyAsync(hb.data(), beta, sizeof(double) * maxm * nt, hipMemcpyDeviceToHost, s));
            DLMA_HIP(hipStreamSynchronize(s));
            // cheap test first: Ritz residual estimates |beta_m s_mi| of the Lanczos operator;
            // at a restart also the kept Ritz pairs and their couplings
            const bool do_restart = restart && m == maxm && !last_step && restarts < max_restarts;
            std::vector<double> Skeep, th_new, sg_new;
            if (do_restart) {
                Skeep.assign((size_t)nt * m * keep, 0.0);
                th_new.assign((size_t)nt * keep, 0.0);
                sg_new.assign((size_t)nt * keep, 0.0);
            }
            std::atomic<bool> trigger(true), solved(true);
            parallel_for(nt, [&](int t) {
                if (!trigger && !do_restart) return true;
                const double bm = hb[(size_t)t * maxm + m - 1];
                std::vector<double> d, Z, last;
                if (!(do_restart ? proj_eig(t, m, d, &Z, nullptr) : proj_eig(t, m, d, nullptr, &last))) {
                    solved = false;
                    return false;
                }
                if (do_restart) last.assign(Z.begin() + (size_t)(m - 1) * m, Z.end());
                std::vector<int> idx = argsort(d);
                if (largest) std::reverse(idx.begin(), idx.end());
                if (bm >= 1e-12)  // else an invariant subspace was reached: Ritz pairs exact
                    for (int k = 0; k < nev; ++k) {
                        double scale = largest ? std::fabs(d[idx[k]]) : 12.0;
                        if (std::fabs(bm * last[idx[k]]) > tol * scale) { trigger = false; break; }
                    }
                if (do_restart)
                    for (int c = 0; c < keep; ++c) {
                        th_new[(size_t)t * keep + c] = d[idx[c]];
                        sg_new[(size_t)t * keep + c] = bm * last[idx[c]];
                        for (int i = 0; i < m; ++i) Skeep[((size_t)t * m + i) * keep + c] = Z[(size_t)i * m + idx[c]];
                    }
                return true;
            });
            if (!solved) return fail(DLMA_EHIP, "projected eigenproblem did not converge");
            if (trigger || last_step || (restart && !do_restart)) {
                bool ok = false;
                DLMA_TRY(ritz_check(m, largest, ok));
                if (ok) { conv = true; return DLMA_OK; }
            }
            if (!do_restart) {
                if (restart) break;  // out of restarts
                continue;
            }
            // restart: q_0..q_{keep-1} = kept Ritz vectors, q_keep = q_m
            Buf Sd;
            DLMA_TRY(Sd.allocate(sizeof(double) * Skeep.size()));
            DLMA_HIP(hipMemcpyAsync(Sd.p, Skeep.data(), sizeof(double) * Skeep.size(), hipMemcpyHostToDevice, s));
            t_begin(ev);
            DLMA_HIP(launch_ritz(q, tsq, isq, Sd.as<double>(), m, keep, RZ.as<double2>(), (long)keep * n, n, nt, s));
            DLMA_HIP(hipMemcpy2DAsync(q, tsq * sizeof(double2), RZ.p, (size_t)keep * n * sizeof(double2),
                                      (size_t)keep * n * sizeof(double2), nt, hipMemcpyDeviceToDevice, s));
            DLMA_HIP(hipMemcpy2DAsync(q + (long)keep * isq, tsq * sizeof(double2), q + (long)m * isq, tsq * sizeof(double2),
                                      n * sizeof(double2), nt, hipMemcpyDeviceToDevice, s));
            t_end(ev, KC_LAP_RITZ, ((double)m + 2.0 * keep + 2.0) * vec_b);
            DLMA_HIP(hipStreamSynchronize(s));  // Skeep's device copy lives in this scope
            theta = std::move(th_new);
            sigma = std::move(sg_new);
            karrow = keep;
            j = keep;
            ++restarts;
        }
        return DLMA_OK;
    };

    int m = 0;
    bool conv = false;
    if (deg > 0) {
        // short unfiltered run: Ritz values are upper bounds of the lowest eigenvalues,
        // so the (nev + nev/4 + 4)-th one lies above every wanted eigenvalue
        int m0 = (int)std::min<long>(std::min(maxm, std::max(2 * nev + 20, 40)), n);
        DLMA_TRY(lanczos(m0, false, false, m, conv, (const double2*)v0));
        DLMA_HIP(hipMemcpyAsync(ha.data(), alpha, sizeof(double) * maxm * nt, hipMemcpyDeviceToHost, s));
        DLMA_HIP(hipMemcpyAsync(hb.data(), beta, sizeof(double) * maxm * nt, hipMemcpyDeviceToHost, s));
        DLMA_HIP(hipStreamSynchronize(s));
        double cut = 0;
        int jc = std::min(m - 1, nev + nev / 4 + 4);
        for (int t = 0; t < nt; ++t) {
            std::vector<double> d(ha.begin() + (size_t)t * maxm, ha.begin() + (size_t)t * maxm + m);
            std::vector<double> e(hb.begin() + (size_t)t * maxm, hb.begin() + (size_t)t * maxm + m - 1);
            if (!tridiag_ql(d, e, nullptr, nullptr)) return fail(DLMA_EHIP, "tridiagonal eigensolver did not converge");
            std::sort(d.begin(), d.end());
            cut = std::max(cut, d[jc]);
        }
        if (cut < 11.0) {  // damp [cut, 12]; otherwise the filter would not help
            cur_deg = deg;
            cc = 0.5 * (cut + 12.0);
            ee = 0.5 * (12.0 - cut);
        }
    }
    // Second estimate of the cut (the final run, thick-restarted or not, keeps it):
    // the unfiltered run's Ritz values lie far above the eigenvalues beyond the wanted
    // ones, so the first cut damps too little of the spectrum.  A short filtered run
    // resolves the top of the filtered spectrum; its (nev + nev/4)-th largest Ritz value
    // theta maps back through the filter to lambda(theta) = c - e cosh(acosh(theta)/deg),
    // an upper bound of that eigenvalue of -lap.  The final run uses the new cut and
    // starts from the sum of the short run's wanted Ritz vectors.
    const double2* start = (const double2*)v0;
    const int mB = (int)std::min<long>(std::min(maxm - 1, nev + std::max(20, nev / 2)), n - 1);
    if (cur_deg > 0 && mB > nev + nev / 4) {
        DLMA_TRY(lanczos(mB, true, false, m, conv, start));
        DLMA_HIP(hipMemcpyAsync(ha.data(), alpha, sizeof(double) * maxm * nt, hipMemcpyDeviceToHost, s));
        DLMA_HIP(hipMemcpyAsync(hb.data(), beta, sizeof(double) * maxm * nt, hipMemcpyDeviceToHost, s));
        DLMA_HIP(hipStreamSynchronize(s));
        double cut2 = 0;
        std::vector<double> Ssum((size_t)nt * m, 0.0);
        bool ok = true;
        for (int t = 0; t < nt && ok; ++t) {
            std::vector<double> d, Z;
            if (!proj_eig(t, m, d, &Z, nullptr)) { ok = false; break; }
            std::vector<int> idx = argsort(d);
            std::reverse(idx.begin(), idx.end());
            const double th = d[idx[nev + nev / 4]];
            const double lam = th > 1.0 ? cc - ee * std::cosh(std::acosh(th) / cur_deg) : 12.0;
            cut2 = std::max(cut2, lam);
            for (int k = 0; k < nev; ++k)
                for (int i = 0; i < m; ++i) Ssum[(size_t)t * m + i] += Z[(size_t)i * m + idx[k]];
        }
        if (!ok) return fail(DLMA_EHIP, "tridiagonal eigensolver did not converge");
        if (cut2 < cc - ee) {  // a lower cut than the first (cc - ee is the current cut)
            cc = 0.5 * (cut2 + 12.0);
            ee = 0.5 * (12.0 - cut2);
        }
        // start vector: q times the summed coefficients (one Ritz combination per timeslice)
        Buf Sd;
        DLMA_TRY(Sd.allocate(sizeof(double) * Ssum.size()));
        DLMA_HIP(hipMemcpyAsync(Sd.p, Ssum.data(), sizeof(double) * Ssum.size(), hipMemcpyHostToDevice, s));
        DLMA_HIP(launch_ritz(q, tsq, isq, Sd.as<double>(), m, 1, AY.as<double2>(), n, n, nt, s));
        DLMA_HIP(hipStreamSynchronize(s));  // Sd's device copy lives in this scope
        start = AY.as<double2>();
    }
    DLMA_TRY(lanczos(restart ? (long)(max_restarts + 1) * maxm : (long)maxm, cur_deg > 0, true, m, conv, start));
    if (!conv) {  // basis cap reached: report the last Ritz pairs
        bool ok = false;
        DLMA_TRY(ritz_check(m, cur_deg > 0, ok));
        conv = ok;
    }
    // order by eigenvalue of -lap (ascending) within each timeslice
    std::vector<int> perm((size_t)nt * nev);
    bool permute = false;
    for (int t = 0; t < nt; ++t) {
        std::vector<double> l(hlam.begin() + (size_t)t * nev, hlam.begin() + (size_t)t * nev + nev);
        std::vector<int> idx = argsort(l);
        for (int k = 0; k < nev; ++k) {
            perm[(size_t)t * nev + k] = idx[k];
            if (idx[k] != k) permute = true;
            evals[(size_t)t * nev + k] = -l[idx[k]];
        }
    }
    if (permute) {
        DLMA_HIP(hipMemcpyAsync(AY.p, Vo, sizeof(double2) * (size_t)nt * nev * n, hipMemcpyDeviceToDevice, s));
        for (int t = 0; t < nt; ++t)
            for (int k = 0; k < nev; ++k)
                DLMA_HIP(hipMemcpyAsync(Vo + ((size_t)t * nev + k) * n, AY.as<double2>() + ((size_t)t * nev + perm[(size_t)t * nev + k]) * n,
                                        sizeof(double2) * n, hipMemcpyDeviceToDevice, s));
    }
    DLMA_HIP(launch_phase_fix(Vo, n, nev * nt, s));
    DLMA_HIP(hipStreamSynchronize(s));
    if (prof.on) prof.collect();
    if (!conv) return fail(DLMA_ENOTCONV, "Lanczos did not reach the tolerance within max_basis steps");
    return DLMA_OK;
}

extern "C" int dlma_dot(const void* a, const void* b, long n, double* out, void* stream) {
    if (!a || !b || !out) return fail(DLMA_EINVAL, "NULL pointer");
    if (n < 0) return fail(DLMA_EINVAL, "n < 0");
    hipStream_t s = S(stream);
    Buf r;
    DLMA_TRY(r.allocate(sizeof(double2)));
    DLMA_HIP(launch_dots((const double2*)a, 0, 0, (const double2*)b, 0, n, r.as<double2>(), 1, 1, 1, s));
    double2 h;
    DLMA_HIP(hipMemcpyAsync(&h, r.p, sizeof(double2), hipMemcpyDeviceToHost, s));
    DLMA_HIP(hipStreamSynchronize(s));
    out[0] = h.x;
    out[1] = h.y;
    return DLMA_OK;
}

extern "C" int dlma_project(dlma_gauge_t h, int t, int nev, const void* V_t, const void* in, void* out, int nrhs, int mode,
                            void* stream) {
    Gauge* g = (Gauge*)h;
    if (!g) return fail(DLMA_EINVAL, "NULL handle");
    if (t < 0 || t >= g->dims[0]) return fail(DLMA_EINVAL, "timeslice out of range");
    if (mode != 0 && mode != 1) return fail(DLMA_EINVAL, "mode must be 0 or 1");
    if (nrhs < 0 || nev < 0) return fail(DLMA_EINVAL, "negative count");
    if (nrhs == 0) return DLMA_OK;
    if (!in || !out || (nev > 0 && !V_t)) return fail(DLMA_EINVAL, "NULL pointer");
    hipStream_t s = S(stream);
    Buf coef;
    DLMA_TRY(coef.allocate(sizeof(double2) * std::max(1, nev) * 4 * (size_t)std::min(nrhs, 65535)));
    DLMA_HIP(launch_project((const double2*)V_t, (const double2*)in, (double2*)out, g->geo, t, nev, nrhs, mode, coef.as<double2>(), s));
    DLMA_HIP(hipStreamSynchronize(s));
    return DLMA_OK;
}

// ---------------------------------------------------------------- correlators

namespace {

struct Gam {
    cplx m[4][4];
};

Gam gmul(const Gam& a, const Gam& b) {
    Gam c;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int k = 0; k < 4; ++k) s += a.m[i][k] * b.m[k][j];
            c.m[i][j] = s;
        }
    return c;
}

// chiral basis: g0 = [[0,-1],[-1,0]], gk = [[0,-i sk],[i sk,0]], g5 = diag(1,1,-1,-1)
std::vector<Gam> gammas() {
    std::vector<Gam> g(5);
    for (auto& x : g)
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) x.m[i][j] = 0;
    const cplx I(0, 1);
    cplx sig[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
    for (int i = 0; i < 2; ++i) {
        g[0].m[i][i + 2] = -1;
        g[0].m[i + 2][i] = -1;
    }
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                g[k + 1].m[i][j + 2] = -I * sig[k][i][j];
                g[k + 1].m[i + 2][j] = I * sig[k][i][j];
            }
    g[4].m[0][0] = g[4].m[1][1] = 1;
    g[4].m[2][2] = g[4].m[3][3] = -1;
    return g;
}

}  // namespace

extern "C" int dlma_correlators(dlma_gauge_t h, int t_src, int nev, const void* V_all, const void* phi_dist, int ndist,
                                int nnoise, int ndil, const void* phi, const void* phibar, double* C_out, void* stream) {
    Gauge* g = (Gauge*)h;
    if (!g) return fail(DLMA_EINVAL, "NULL handle");
    const int T = g->dims[0];
    if (t_src < 0 || t_src >= T) return fail(DLMA_EINVAL, "t_src out of range");
    if (nev < 1 || nnoise < 0 || ndist < 0) return fail(DLMA_EINVAL, "nev must be >= 1, ndist and nnoise >= 0");
    if (ndil < 1 || nnoise % ndil != 0) return fail(DLMA_EINVAL, "ndil must be >= 1 and divide nnoise");
    const double nvec = nnoise > 0 ? (double)(nnoise / ndil) : 1.0;  // independent noise vectors
    if (!V_all || !C_out || (ndist > 0 && !phi_dist) || (nnoise > 0 && (!phi || !phibar)))
        return fail(DLMA_EINVAL, "NULL pointer");
    hipStream_t s = S(stream);
    const long V = g->V;
    const long fs = V * 12;  // complex numbers per spinor field
    const int nd = 4 * ndist, nn = 4 * nnoise;
    // fields: dist solutions, then phi, then phibar
    std::vector<const double2*> fields;
    for (int i = 0; i < nd; ++i) fields.push_back((const double2*)phi_dist + i * fs);
    for (int i = 0; i < nn; ++i) fields.push_back((const double2*)phi + i * fs);
    for (int i = 0; i < nn; ++i) fields.push_back((const double2*)phibar + i * fs);
    const int nf = (int)fields.size();
    // Gram pairs: dist (phi_{l,s'}, phi_{l,s}); noise (phi_{r,s'}, phi_{r,s}) and (phibar_{r,s'}, phi_{r,s})
    std::vector<const double2*> pa, pb;
    for (int l = 0; l < ndist; ++l)
        for (int sp = 0; sp < 4; ++sp)
            for (int sq = 0; sq < 4; ++sq) { pa.push_back(fields[l * 4 + sp]); pb.push_back(fields[l * 4 + sq]); }
    for (int r = 0; r < nnoise; ++r)
        for (int y = 0; y < 2; ++y)
            for (int sp = 0; sp < 4; ++sp)
                for (int sq = 0; sq < 4; ++sq) {
                    pa.push_back(fields[nd + (y ? nn : 0) + r * 4 + sp]);
                    pb.push_back(fields[nd + r * 4 + sq]);
                }
    const int np = (int)pa.size();
    Buf dF, dA, dB, dP, dG;
    DLMA_TRY(dF.allocate(sizeof(void*) * std::max(1, nf)));
    DLMA_TRY(dA.allocate(sizeof(void*) * std::max(1, np)));
    DLMA_TRY(dB.allocate(sizeof(void*) * std::max(1, np)));
    DLMA_TRY(dP.allocate(sizeof(double2) * (size_t)nf * T * nev * 4));
    DLMA_TRY(dG.allocate(sizeof(double2) * (size_t)np * T * 16));
    DLMA_HIP(hipMemcpyAsync(dF.p, fields.data(), sizeof(void*) * nf, hipMemcpyHostToDevice, s));
    DLMA_HIP(hipMemcpyAsync(dA.p, pa.data(), sizeof(void*) * np, hipMemcpyHostToDevice, s));
    DLMA_HIP(hipMemcpyAsync(dB.p, pb.data(), sizeof(void*) * np, hipMemcpyHostToDevice, s));
    DLMA_HIP(launch_tproj((const double2*)V_all, (const double2* const*)dF.p, nf, g->geo, nev, dP.as<double2>(), s));
    DLMA_HIP(launch_spin_gram((const double2* const*)dA.p, (const double2* const*)dB.p, np, g->geo, dG.as<double2>(), s));
    std::vector<cplx> P((size_t)nf * T * nev * 4), G((size_t)np * T * 16);
    DLMA_HIP(hipMemcpyAsync(P.data(), dP.p, sizeof(double2) * P.size(), hipMemcpyDeviceToHost, s));
    DLMA_HIP(hipMemcpyAsync(G.data(), dG.p, sizeof(double2) * G.size(), hipMemcpyDeviceToHost, s));
    DLMA_HIP(hipStreamSynchronize(s));

    // Host assembly of the few numbers per timeslice from the GPU projections and Grams.
    auto Pf = [&](int f, int t, int k, int sp) { return P[(((size_t)f * T + t) * nev + k) * 4 + sp]; };
    auto Gp = [&](int p, int t, int s1, int s2) { return G[((size_t)p * T + t) * 16 + s1 * 4 + s2]; };
    std::vector<Gam> ga = gammas();
    const Gam g5 = ga[4];
    std::fill(C_out, C_out + (size_t)DLMA_NGAMMA * DLMA_NPARTS * T * 2, 0.0);
    for (int gi = 0; gi < DLMA_NGAMMA; ++gi) {
        std::vector<Gam> Gs;
        if (gi == 0) Gs.push_back(g5);
        else Gs = {ga[1], ga[2], ga[3]};
        std::vector<cplx> acc((size_t)DLMA_NPARTS * T, 0.0);
        for (const Gam& Gm : Gs) {
            Gam M = gmul(g5, Gm), N = gmul(Gm, g5);
            for (int d = 0; d < T; ++d) {
                int t = (t_src + d) % T;
                // <A, M B>_t from a Gram, <A, M P_t B>_t from projections
                auto mg = [&](int p) {
                    cplx v = 0;
                    for (int a = 0; a < 4; ++a)
                        for (int b = 0; b < 4; ++b)
                            if (M.m[a][b] != 0.0) v += M.m[a][b] * Gp(p, t, a, b);
                    return v;
                };
                auto mp = [&](int fa, int fb) {
                    cplx v = 0;
                    for (int k = 0; k < nev; ++k)
                        for (int a = 0; a < 4; ++a)
                            for (int b = 0; b < 4; ++b)
                                if (M.m[a][b] != 0.0) v += M.m[a][b] * std::conj(Pf(fa, t, k, a)) * Pf(fb, t, k, b);
                    return v;
                };
                // noise estimators
                if (nnoise > 0) {
                    cplx qq = 0, pq = 0, qp = 0, pp = 0, one = 0;
                    for (int r = 0; r < nnoise; ++r)
                        for (int s1 = 0; s1 < 4; ++s1)       // s: source spin of phi_{r,s}
                            for (int s2 = 0; s2 < 4; ++s2) {  // s': spin of phiY_{r,s'}
                                cplx nc = N.m[s1][s2];
                                if (nc == 0.0) continue;
                                int p1 = ndist * 16 + (r * 2 + 0) * 16 + s2 * 4 + s1;  // (phi_{r,s'}, phi_{r,s})
                                int pQ = ndist * 16 + (r * 2 + 1) * 16 + s2 * 4 + s1;  // (phibar_{r,s'}, phi_{r,s})
                                int fB = nd + r * 4 + s1;
                                int fA1 = nd + r * 4 + s2, fAQ = nd + nn + r * 4 + s2;
                                cplx g1 = mg(p1), gQ = mg(pQ);
                                cplx P1 = mp(fA1, fB), PQ = mp(fAQ, fB);
                                // Y = 1: phi; Y = Q: phibar; Y = P: phi - phibar.  X = P: projected; Q = 1 - P
                                cplx y1x1 = g1, y1xp = P1, yqx1 = gQ, yqxp = PQ;
                                cplx ypx1 = g1 - gQ, ypxp = P1 - PQ;
                                qq += nc * (yqx1 - yqxp);
                                pq += nc * yqxp;
                                qp += nc * (ypx1 - ypxp);
                                pp += nc * ypxp;
                                one += nc * y1x1;
                                (void)y1xp;
                            }
                    acc[0 * T + d] += qq / nvec;
                    acc[1 * T + d] += pq / nvec;
                    acc[2 * T + d] += qp / nvec;
                    acc[3 * T + d] += pp / nvec;
                    acc[4 * T + d] += one / nvec;
                }
                // exact C_dist from the perambulator tau_{(k s),(l s')} = P[l*4+s'][t][k][s]
                cplx cd = 0;
                for (int k = 0; k < nev; ++k)
                    for (int l = 0; l < ndist; ++l)
                        for (int s1 = 0; s1 < 4; ++s1)
                            for (int s2 = 0; s2 < 4; ++s2) {
                                if (M.m[s1][s2] == 0.0) continue;
                                for (int s3 = 0; s3 < 4; ++s3)
                                    for (int s4 = 0; s4 < 4; ++s4) {
                                        if (N.m[s3][s4] == 0.0) continue;
                                        cd += M.m[s1][s2] * Pf(l * 4 + s3, t, k, s2) * N.m[s3][s4] * std::conj(Pf(l * 4 + s4, t, k, s1));
                                    }
                            }
                acc[5 * T + d] += cd;
                // exact C_QP from the distillation solutions
                cplx cq = 0;
                for (int l = 0; l < ndist; ++l)
                    for (int s1 = 0; s1 < 4; ++s1)
                        for (int s2 = 0; s2 < 4; ++s2) {
                            cplx nc = N.m[s1][s2];
                            if (nc == 0.0) continue;
                            int p = l * 16 + s2 * 4 + s1;  // (phi_{l,s'}, phi_{l,s})
                            cq += nc * (mg(p) - mp(l * 4 + s2, l * 4 + s1));
                        }
                acc[6 * T + d] += cq;
            }
        }
        for (int part = 0; part < DLMA_NPARTS; ++part)
            for (int d = 0; d < T; ++d) {
                cplx v = acc[(size_t)part * T + d] / (double)Gs.size();
                C_out[(((size_t)gi * DLMA_NPARTS + part) * T + d) * 2 + 0] = v.real();
                C_out[(((size_t)gi * DLMA_NPARTS + part) * T + d) * 2 + 1] = v.imag();
            }
    }
    return DLMA_OK;
}

// Backward of dlma_correlators.  Each piece is
//   c / |Gamma list| sum_Gamma sum_grp sum_{s,s'} N_{s s'} <A_{grp,s'}, M X_t B_{grp,s}>_t,
// M = g5 Gamma, N = Gamma g5, X in {1, box, 1 - box}, so a real loss with weights G on
// the pieces (dL/dRe C + i dL/dIm C) has the gradient fields
//   grad B_{grp,s}  += w(t) conj(N_{s s'}) X_t M^dag A_{grp,s'},
//   grad A_{grp,s'} += conj(w(t)) N_{s s'} M X_t B_{grp,s},     w = G c / |Gamma list|.
// The host folds every piece, Gamma and sign into two matrices per timeslice over the
// (field, spin) components of one source group, W1 (X = 1 parts) and WP (box parts;
// 1 - box splits into both), shared by all groups; the kernel forms W1 F + box(t) WP F
// with box(t) WP F = sum_k v_k(t) (WP V(t)^dag F)_k.
extern "C" int dlma_correlators_grad(dlma_gauge_t h, int t_src, int nev, const void* V_all, const void* phi_dist, int ndist,
                                     int nnoise, int ndil, const void* phi, const void* phibar, const double* G_in,
                                     void* grad_dist, void* grad_phi, void* grad_phibar, void* stream) {
    Gauge* g = (Gauge*)h;
    if (!g) return fail(DLMA_EINVAL, "NULL handle");
    const int T = g->dims[0];
    if (t_src < 0 || t_src >= T) return fail(DLMA_EINVAL, "t_src out of range");
    if (nev < 1 || nnoise < 0 || ndist < 0) return fail(DLMA_EINVAL, "nev must be >= 1, ndist and nnoise >= 0");
    if (ndil < 1 || nnoise % ndil != 0) return fail(DLMA_EINVAL, "ndil must be >= 1 and divide nnoise");
    if (2L * nnoise + ndist > 65535) return fail(DLMA_EINVAL, "2 nnoise + ndist must be below 65536");
    if (!V_all || !G_in || (ndist > 0 && (!phi_dist || !grad_dist)) || (nnoise > 0 && (!phi || !phibar || !grad_phi || !grad_phibar)))
        return fail(DLMA_EINVAL, "NULL pointer");
    if (ndist == 0 && nnoise == 0) return DLMA_OK;
    hipStream_t s = S(stream);
    const long L3 = (long)g->dims[1] * g->dims[2] * g->dims[3];
    const long fs = g->V * 12;
    const int nd = 4 * ndist, nn = 4 * nnoise, nf = nd + 2 * nn;
    const double nvec = nnoise > 0 ? (double)(nnoise / ndil) : 1.0;

    // weight matrices per timeslice: noise [T][32][32] over (phi_s, phibar_s) x spin, dist [T][16][16]
    std::vector<cplx> W1n((size_t)T * 1024, 0.0), WPn((size_t)T * 1024, 0.0), W1d((size_t)T * 256, 0.0), WPd((size_t)T * 256, 0.0);
    std::vector<int> tact(T, -1);
    std::vector<Gam> ga = gammas();
    const Gam g5 = ga[4];
    // piece -> X (0: 1, 1: box, 2: 1 - box), source-side field A (0: phibar, 1: phi - phibar, 2: phi, 3: dist)
    const int PX[DLMA_NPARTS] = {2, 1, 2, 1, 0, 1, 2};
    const int PA[DLMA_NPARTS] = {0, 0, 1, 1, 2, 3, 3};
    auto addw = [&](bool dist, int t, int row, int col, cplx v, int X) {
        std::vector<cplx>& W1 = dist ? W1d : W1n;
        std::vector<cplx>& WP = dist ? WPd : WPn;
        const int n = dist ? 16 : 32;
        const size_t i = ((size_t)t * n + row) * n + col;
        if (X != 1) W1[i] += v;       // X = 1 or 1 - box
        if (X == 1) WP[i] += v;       // box
        if (X == 2) WP[i] -= v;       // the box part of 1 - box
    };
    for (int gi = 0; gi < DLMA_NGAMMA; ++gi) {
        std::vector<Gam> Gs;
        if (gi == 0) Gs.push_back(g5);
        else Gs = {ga[1], ga[2], ga[3]};
        for (int part = 0; part < DLMA_NPARTS; ++part) {
            const bool dist = PA[part] == 3;
            if (dist ? ndist == 0 : nnoise == 0) continue;
            const double c = (dist ? 1.0 : 1.0 / nvec) / (double)Gs.size();
            for (int d = 0; d < T; ++d) {
                const double* gp = G_in + (((size_t)gi * DLMA_NPARTS + part) * T + d) * 2;
                const cplx w = cplx(gp[0], gp[1]) * c;
                if (w == 0.0) continue;
                if (!std::isfinite(w.real()) || !std::isfinite(w.imag())) return fail(DLMA_EINVAL, "non-finite weight");
                const int t = (t_src + d) % T;
                tact[t] = 0;
                const int X = PX[part];
                for (const Gam& Gm : Gs) {
                    const Gam M = gmul(g5, Gm), N = gmul(Gm, g5);
                    for (int sg = 0; sg < 4; ++sg)       // s: spin label of B (sink solution)
                        for (int sq = 0; sq < 4; ++sq) {  // s': spin label of A (source-side solution)
                            const cplx nss = N.m[sg][sq];
                            if (nss == 0.0) continue;
                            // A as input columns / output rows: (field index in the group, coefficient)
                            int aj[2];
                            double ac[2];
                            int na = 0;
                            if (dist) { aj[na] = sq; ac[na++] = 1.0; }
                            else if (PA[part] == 0) { aj[na] = 4 + sq; ac[na++] = 1.0; }
                            else if (PA[part] == 1) { aj[na] = sq; ac[na++] = 1.0; aj[na] = 4 + sq; ac[na++] = -1.0; }
                            else { aj[na] = sq; ac[na++] = 1.0; }
                            const cplx cb = w * std::conj(nss);  // grad B_s += cb X M^dag A_s'
                            const cplx ca = std::conj(w) * nss;  // grad A_s' += ca M X B_s
                            for (int a = 0; a < 4; ++a)
                                for (int b = 0; b < 4; ++b) {
                                    const cplx mdag = std::conj(M.m[b][a]), m = M.m[a][b];
                                    for (int q = 0; q < na; ++q) {
                                        if (mdag != 0.0) addw(dist, t, sg * 4 + a, aj[q] * 4 + b, cb * ac[q] * mdag, X);
                                        if (m != 0.0) addw(dist, t, aj[q] * 4 + a, sg * 4 + b, ca * ac[q] * m, X);
                                    }
                                }
                        }
                }
            }
        }
    }
    int nact = 0;
    for (int t = 0; t < T; ++t)
        if (tact[t] >= 0) tact[t] = nact++;
    // projections of every input field on the modes of every timeslice: P[f][t][k][s]
    std::vector<const double2*> fields;
    for (int i = 0; i < nd; ++i) fields.push_back((const double2*)phi_dist + i * fs);
    for (int i = 0; i < nn; ++i) fields.push_back((const double2*)phi + i * fs);
    for (int i = 0; i < nn; ++i) fields.push_back((const double2*)phibar + i * fs);
    Buf dF, dP, dW1n, dW1d, dTn, dTd, dTact;
    std::vector<cplx> P;
    if (nact > 0) {
        DLMA_TRY(dF.allocate(sizeof(void*) * nf));
        DLMA_TRY(dP.allocate(sizeof(double2) * (size_t)nf * T * nev * 4));
        DLMA_HIP(hipMemcpyAsync(dF.p, fields.data(), sizeof(void*) * nf, hipMemcpyHostToDevice, s));
        DLMA_HIP(launch_tproj((const double2*)V_all, (const double2* const*)dF.p, nf, g->geo, nev, dP.as<double2>(), s));
        P.resize((size_t)nf * T * nev * 4);
        DLMA_HIP(hipMemcpyAsync(P.data(), dP.p, sizeof(double2) * P.size(), hipMemcpyDeviceToHost, s));
        DLMA_HIP(hipStreamSynchronize(s));
    }
    // tau' = WP(t) tau for every group and weighted timeslice
    std::vector<cplx> taun((size_t)std::max(1, nnoise) * std::max(1, nact) * nev * 32, 0.0);
    std::vector<cplx> taud((size_t)std::max(1, ndist) * std::max(1, nact) * nev * 16, 0.0);
    auto Pf = [&](int f, int t, int k, int sp) { return P[(((size_t)f * T + t) * nev + k) * 4 + sp]; };
    for (int t = 0; t < T; ++t) {
        const int ta = tact[t];
        if (ta < 0) continue;
        for (int r = 0; r < nnoise; ++r)
            for (int k = 0; k < nev; ++k)
                for (int row = 0; row < 32; ++row) {
                    cplx v = 0;
                    for (int col = 0; col < 32; ++col) {
                        const cplx wv = WPn[((size_t)t * 32 + row) * 32 + col];
                        if (wv == 0.0) continue;
                        const int j = col >> 2, b = col & 3;
                        const int f = j < 4 ? nd + r * 4 + j : nd + nn + r * 4 + (j - 4);
                        v += wv * Pf(f, t, k, b);
                    }
                    taun[(((size_t)r * nact + ta) * nev + k) * 32 + row] = v;
                }
        for (int l = 0; l < ndist; ++l)
            for (int k = 0; k < nev; ++k)
                for (int row = 0; row < 16; ++row) {
                    cplx v = 0;
                    for (int col = 0; col < 16; ++col) {
                        const cplx wv = WPd[((size_t)t * 16 + row) * 16 + col];
                        if (wv == 0.0) continue;
                        v += wv * Pf(l * 4 + (col >> 2), t, k, col & 3);
                    }
                    taud[(((size_t)l * nact + ta) * nev + k) * 16 + row] = v;
                }
    }
    DLMA_TRY(dW1n.allocate(sizeof(double2) * W1n.size()));
    DLMA_TRY(dW1d.allocate(sizeof(double2) * W1d.size()));
    DLMA_TRY(dTn.allocate(sizeof(double2) * taun.size()));
    DLMA_TRY(dTd.allocate(sizeof(double2) * taud.size()));
    DLMA_TRY(dTact.allocate(sizeof(int) * T));
    DLMA_HIP(hipMemcpyAsync(dW1n.p, W1n.data(), sizeof(double2) * W1n.size(), hipMemcpyHostToDevice, s));
    DLMA_HIP(hipMemcpyAsync(dW1d.p, W1d.data(), sizeof(double2) * W1d.size(), hipMemcpyHostToDevice, s));
    DLMA_HIP(hipMemcpyAsync(dTn.p, taun.data(), sizeof(double2) * taun.size(), hipMemcpyHostToDevice, s));
    DLMA_HIP(hipMemcpyAsync(dTd.p, taud.data(), sizeof(double2) * taud.size(), hipMemcpyHostToDevice, s));
    DLMA_HIP(hipMemcpyAsync(dTact.p, tact.data(), sizeof(int) * T, hipMemcpyHostToDevice, s));
    CorrGradArgs a = {};
    a.Vall = (const double2*)V_all;
    a.dist = (const double2*)phi_dist; a.phi = (const double2*)phi; a.phibar = (const double2*)phibar;
    a.gdist = (double2*)grad_dist; a.gphi = (double2*)grad_phi; a.gphibar = (double2*)grad_phibar;
    a.W1n = dW1n.as<double2>(); a.W1d = dW1d.as<double2>();
    a.taun = dTn.as<double2>(); a.taud = dTd.as<double2>();
    a.tact = dTact.as<int>();
    a.L3 = L3; a.fs = fs; a.nev = nev; a.ndist = ndist; a.nnoise = nnoise; a.nact = std::max(1, nact);
    DLMA_HIP(launch_corr_grad(a, T, s));
    DLMA_HIP(hipStreamSynchronize(s));  // the host tables are released on return
    return DLMA_OK;
}
