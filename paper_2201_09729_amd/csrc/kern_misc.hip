// Gauge packing, clover construction and inversion, layout conversions, site-local
// vector kernels and the fixed-order reduction finishers.
#include "kernels.h"

namespace dlma {

// ---------------------------------------------------------------- helpers

struct C64 { double r, i; };
HD C64 cmul(C64 a, C64 b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
HD C64 cadd(C64 a, C64 b) { return {a.r + b.r, a.i + b.i}; }
HD C64 cconj(C64 a) { return {a.r, -a.i}; }

struct M3 { C64 m[9]; };

HD M3 ldU(const double2* U, long site, int mu) {
    M3 o;
    const double2* p = U + (site * 4 + mu) * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) { double2 v = p[k]; o.m[k] = {v.x, v.y}; }
    return o;
}
HD M3 dagm(const M3& a) {
    M3 o;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) o.m[i * 3 + j] = cconj(a.m[j * 3 + i]);
    return o;
}
HD M3 mulm(const M3& a, const M3& b) {
    M3 o;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            C64 s = {0, 0};
#pragma unroll
            for (int k = 0; k < 3; ++k) s = cadd(s, cmul(a.m[i * 3 + k], b.m[k * 3 + j]));
            o.m[i * 3 + j] = s;
        }
    return o;
}

struct Coord { int c[4]; };  // c[mu], mu = 0:t 1:x 2:y 3:z

HD Coord coord_of(const Geo& g, long s) {
    Coord o;
    o.c[1] = (int)(s % g.X); s /= g.X;
    o.c[2] = (int)(s % g.Y); s /= g.Y;
    o.c[3] = (int)(s % g.Z); s /= g.Z;
    o.c[0] = (int)s;
    return o;
}
HD int ext(const Geo& g, int mu) { return mu == 0 ? g.T : (mu == 1 ? g.X : (mu == 2 ? g.Y : g.Z)); }
HD long site_of(const Geo& g, Coord c) {
    return (((long)c.c[0] * g.Z + c.c[3]) * g.Y + c.c[2]) * g.X + c.c[1];
}
HD Coord shift(const Geo& g, Coord c, int mu, int d) {
    int L = ext(g, mu);
    c.c[mu] = (c.c[mu] + d + L) % L;
    return c;
}

// ---------------------------------------------------------------- gauge packing

__global__ void k_pack_links(const double2* __restrict__ Ucan, double2* __restrict__ U64, Geo g) {
    long V = 2L * g.Vh;
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V * 4) return;
    long s = i >> 2;
    int mu = (int)(i & 3);
    Coord c = coord_of(g, s);
    int par = (c.c[0] + c.c[1] + c.c[2] + c.c[3]) & 1;
    long cb = s >> 1;  // ((t*Z+z)*Y+y)*Xh + x/2 since X is even
    for (int k = 0; k < 9; ++k) U64[((size_t)(par * 4 + mu) * 9 + k) * g.Vh + cb] = Ucan[(s * 4 + mu) * 9 + k];
}

hipError_t launch_pack_links(const double2* Ucan, double2* U64, const Geo& g, hipStream_t s) {
    long n = 2L * g.Vh * 4;
    hipLaunchKernelGGL(k_pack_links, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Ucan, U64, g);
    return hipGetLastError();
}

// per block: max over its links of max_ij |(U U^dag - 1)_ij| (NaN propagates as +inf)
__global__ void k_unitarity(const double2* __restrict__ Ucan, long nlink, double* __restrict__ blockmax) {
    __shared__ double sm[256];
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double m = 0.0;
    if (i < nlink) {
        M3 u;
#pragma unroll
        for (int k = 0; k < 9; ++k) { double2 v = Ucan[i * 9 + k]; u.m[k] = {v.x, v.y}; }
        M3 p = mulm(u, dagm(u));
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double re = p.m[a * 3 + b].r - (a == b ? 1.0 : 0.0), im = p.m[a * 3 + b].i;
                double e = fabs(re) + fabs(im);
                if (!(e == e) || isinf(e)) e = INFINITY;
                m = fmax(m, e);
            }
    }
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) blockmax[blockIdx.x] = sm[0];
}

hipError_t launch_unitarity(const double2* Ucan, long nlink, double* blockmax, int nblk, hipStream_t s) {
    hipLaunchKernelGGL(k_unitarity, dim3(nblk), dim3(256), 0, s, Ucan, nlink, blockmax);
    return hipGetLastError();
}

// ---------------------------------------------------------------- clover

// Four-leaf clover Q_{mu nu}(x): the four plaquettes of the (mu,nu) plane touching x,
// each traversed counter-clockwise from x.
HD M3 leaves(const double2* U, const Geo& g, Coord x, int mu, int nu) {
    long sx = site_of(g, x);
    Coord xpm = shift(g, x, mu, 1), xpn = shift(g, x, nu, 1);
    Coord xmm = shift(g, x, mu, -1), xmn = shift(g, x, nu, -1);
    Coord xmm_pn = shift(g, xmm, nu, 1), xmm_mn = shift(g, xmm, nu, -1), xmn_pm = shift(g, xmn, mu, 1);
    long s_pm = site_of(g, xpm), s_pn = site_of(g, xpn), s_mm = site_of(g, xmm), s_mn = site_of(g, xmn);
    long s_mmpn = site_of(g, xmm_pn), s_mmmn = site_of(g, xmm_mn), s_mnpm = site_of(g, xmn_pm);
    M3 Q;
    M3 t = mulm(mulm(ldU(U, sx, mu), ldU(U, s_pm, nu)), mulm(dagm(ldU(U, s_pn, mu)), dagm(ldU(U, sx, nu))));
    Q = t;
    t = mulm(mulm(ldU(U, sx, nu), dagm(ldU(U, s_mmpn, mu))), mulm(dagm(ldU(U, s_mm, nu)), ldU(U, s_mm, mu)));
    for (int k = 0; k < 9; ++k) Q.m[k] = cadd(Q.m[k], t.m[k]);
    t = mulm(mulm(dagm(ldU(U, s_mm, mu)), dagm(ldU(U, s_mmmn, nu))), mulm(ldU(U, s_mmmn, mu), ldU(U, s_mn, nu)));
    for (int k = 0; k < 9; ++k) Q.m[k] = cadd(Q.m[k], t.m[k]);
    t = mulm(mulm(dagm(ldU(U, s_mn, nu)), ldU(U, s_mn, mu)), mulm(ldU(U, s_mnpm, nu), dagm(ldU(U, sx, mu))));
    for (int k = 0; k < 9; ++k) Q.m[k] = cadd(Q.m[k], t.m[k]);
    return Q;
}

// A(x) in the chiral basis splits into two 6x6 blocks (spins 0,1 and spins 2,3):
//   block = (4+m0) 1 + csw (i/2) [[B3, B1 - i B2], [B1 + i B2, -B3]]  (2x2 in spin, 3x3 in colour)
// upper: B1 = F01 - F23, B2 = F02 + F13, B3 = F03 - F12
// lower: B1 = -F01 - F23, B2 = -F02 + F13, B3 = -F03 - F12
// (from sigma_0k = diag(sk, -sk) and sigma_jk = -eps_jkl diag(sl, sl) in this basis).
HD void clover_site(const double2* U, const Geo& g, double m0, double csw, double2* C0, double2* C1, long s) {
    Coord x = coord_of(g, s);
    M3 F[6];
    int p = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu, ++p) {
            M3 Q = leaves(U, g, x, mu, nu);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    C64 q = Q.m[a * 3 + b], qt = cconj(Q.m[b * 3 + a]);
                    F[p].m[a * 3 + b] = {(q.r - qt.r) / 8.0, (q.i - qt.i) / 8.0};
                }
        }
    // planes: 0:01 1:02 2:03 3:12 4:13 5:23
    int par = (x.c[0] + x.c[1] + x.c[2] + x.c[3]) & 1;
    long cb = s >> 1;
    double2* C = par ? C1 : C0;
    for (int blk = 0; blk < 2; ++blk) {
        double sg = blk == 0 ? 1.0 : -1.0;
        C64 B[3][9];
        for (int k = 0; k < 9; ++k) {
            B[0][k] = {sg * F[0].m[k].r - F[5].m[k].r, sg * F[0].m[k].i - F[5].m[k].i};
            B[1][k] = {sg * F[1].m[k].r + F[4].m[k].r, sg * F[1].m[k].i + F[4].m[k].i};
            B[2][k] = {sg * F[2].m[k].r - F[3].m[k].r, sg * F[2].m[k].i - F[3].m[k].i};
        }
        // full 6x6: index i = s*3 + a
        C64 H[36];
        for (int s1 = 0; s1 < 2; ++s1)
            for (int s2 = 0; s2 < 2; ++s2)
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        int k = a * 3 + b;
                        C64 v;
                        if (s1 == 0 && s2 == 0) v = B[2][k];
                        else if (s1 == 1 && s2 == 1) v = {-B[2][k].r, -B[2][k].i};
                        else if (s1 == 0) v = {B[0][k].r + B[1][k].i, B[0][k].i - B[1][k].r};  // B1 - i B2
                        else v = {B[0][k].r - B[1][k].i, B[0][k].i + B[1][k].r};               // B1 + i B2
                        // csw (i/2) v
                        C64 w = {-0.5 * csw * v.i, 0.5 * csw * v.r};
                        if (s1 == s2 && a == b) w.r += 4.0 + m0;
                        H[(s1 * 3 + a) * 6 + s2 * 3 + b] = w;
                    }
        double2* o = C + (size_t)blk * 18 * g.Vh + cb;
        o[0 * (size_t)g.Vh] = make_double2(H[0].r, H[7].r);
        o[1 * (size_t)g.Vh] = make_double2(H[14].r, H[21].r);
        o[2 * (size_t)g.Vh] = make_double2(H[28].r, H[35].r);
        int q = 3;
        for (int i = 1; i < 6; ++i)
            for (int j = 0; j < i; ++j, ++q) o[(size_t)q * g.Vh] = make_double2(H[i * 6 + j].r, H[i * 6 + j].i);
    }
}

__global__ void k_clover_build(const double2* __restrict__ U, Geo g, double m0, double csw,
                               double2* __restrict__ C0, double2* __restrict__ C1) {
    long V = 2L * g.Vh;
    long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    clover_site(U, g, m0, csw, C0, C1, s);
}

hipError_t launch_clover_build(const double2* Ucan, const Geo& g, double m0, double csw, double2* C0, double2* C1, hipStream_t s) {
    long n = 2L * g.Vh;
    hipLaunchKernelGGL(k_clover_build, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, Ucan, g, m0, csw, C0, C1);
    return hipGetLastError();
}

// Inverse of one packed Hermitian positive definite 6x6 block by Cholesky:
// H = L L^dag, M = L^-1, H^-1 = M^dag M.  *err is set if a pivot is not positive.
HD bool clover_invert_block(const double2* C, double2* Ci, int Vh, long i) {
    int blk = (int)(i / Vh);
    long cb = i - (long)blk * Vh;
    const double2* src = C + (size_t)blk * 18 * Vh + cb;
    C64 H[36];
    double2 d0 = src[0], d1 = src[(size_t)Vh], d2 = src[2 * (size_t)Vh];
    double dg[6] = {d0.x, d0.y, d1.x, d1.y, d2.x, d2.y};
    for (int a = 0; a < 6; ++a) H[a * 6 + a] = {dg[a], 0.0};
    int q = 3;
    for (int a = 1; a < 6; ++a)
        for (int b = 0; b < a; ++b, ++q) {
            double2 v = src[(size_t)q * Vh];
            H[a * 6 + b] = {v.x, v.y};
            H[b * 6 + a] = {v.x, -v.y};
        }
    C64 L[36];
    for (int k = 0; k < 36; ++k) L[k] = {0, 0};
    bool ok = true;
    for (int j = 0; j < 6; ++j) {
        double s = H[j * 6 + j].r;
        for (int k = 0; k < j; ++k) s -= L[j * 6 + k].r * L[j * 6 + k].r + L[j * 6 + k].i * L[j * 6 + k].i;
        if (!(s > 0.0)) { ok = false; s = 1.0; }
        double ljj = sqrt(s);
        L[j * 6 + j] = {ljj, 0};
        for (int a = j + 1; a < 6; ++a) {
            C64 t = H[a * 6 + j];
            for (int k = 0; k < j; ++k) {
                C64 p = cmul(L[a * 6 + k], cconj(L[j * 6 + k]));
                t.r -= p.r; t.i -= p.i;
            }
            L[a * 6 + j] = {t.r / ljj, t.i / ljj};
        }
    }
    // M = L^-1 (lower triangular)
    C64 M[36];
    for (int k = 0; k < 36; ++k) M[k] = {0, 0};
    for (int a = 0; a < 6; ++a) {
        M[a * 6 + a] = {1.0 / L[a * 6 + a].r, 0};
        for (int b = a - 1; b >= 0; --b) {
            // M[a][b] = -(sum_{k=b}^{a-1} L[a][k] M[k][b]) / L[a][a]
            C64 s = {0, 0};
            for (int k = b; k < a; ++k) s = cadd(s, cmul(L[a * 6 + k], M[k * 6 + b]));
            M[a * 6 + b] = {-s.r / L[a * 6 + a].r, -s.i / L[a * 6 + a].r};
        }
    }
    // Hinv[a][b] = sum_{k >= max(a,b)} conj(M[k][a]) M[k][b]
    double2* dst = Ci + (size_t)blk * 18 * Vh + cb;
    double dd[6];
    for (int a = 0; a < 6; ++a) {
        double s = 0;
        for (int k = a; k < 6; ++k) s += M[k * 6 + a].r * M[k * 6 + a].r + M[k * 6 + a].i * M[k * 6 + a].i;
        dd[a] = s;
    }
    dst[0] = make_double2(dd[0], dd[1]);
    dst[(size_t)Vh] = make_double2(dd[2], dd[3]);
    dst[2 * (size_t)Vh] = make_double2(dd[4], dd[5]);
    q = 3;
    for (int a = 1; a < 6; ++a)
        for (int b = 0; b < a; ++b, ++q) {
            C64 s = {0, 0};
            for (int k = a; k < 6; ++k) s = cadd(s, cmul(cconj(M[k * 6 + a]), M[k * 6 + b]));
            dst[(size_t)q * Vh] = make_double2(s.r, s.i);
        }
    return ok;
}

__global__ void k_clover_invert(const double2* __restrict__ C, double2* __restrict__ Ci, int Vh, int* err) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2L * Vh) return;
    if (!clover_invert_block(C, Ci, Vh, i)) atomicOr(err, 1);
}

hipError_t launch_clover_invert(const double2* C, double2* Ci, int Vh, int* err, hipStream_t s) {
    long n = 2L * Vh;
    hipLaunchKernelGGL(k_clover_invert, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, C, Ci, Vh, err);
    return hipGetLastError();
}

__global__ void k_add_diag(double2* C, int Vh, double delta) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2L * Vh) return;
    int blk = (int)(i / Vh);
    long cb = i - (long)blk * Vh;
    for (int q = 0; q < 3; ++q) {
        double2* p = C + ((size_t)blk * 18 + q) * Vh + cb;
        double2 v = *p;
        v.x += delta;
        v.y += delta;
        *p = v;
    }
}

hipError_t launch_add_diag(double2* C, int Vh, double delta, hipStream_t s) {
    long n = 2L * Vh;
    hipLaunchKernelGGL(k_add_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C, Vh, delta);
    return hipGetLastError();
}

template <int P> __global__ void k_convert_pairs(const double2* __restrict__ src, typename PT<P>::S* __restrict__ dst, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 v = src[i];
    stp<P>(dst, i, (typename PT<P>::R)v.x, (typename PT<P>::R)v.y);
}

template <int P> hipError_t launch_convert_pairs(const double2* src, void* dst, long n, hipStream_t s) {
    hipLaunchKernelGGL(k_convert_pairs<P>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, (typename PT<P>::S*)dst, n);
    return hipGetLastError();
}
template hipError_t launch_convert_pairs<P32>(const double2*, void*, long, hipStream_t);
template hipError_t launch_convert_pairs<P16>(const double2*, void*, long, hipStream_t);
template hipError_t launch_convert_pairs<PB16>(const double2*, void*, long, hipStream_t);

// FP64 pairs in planes [M][K][Vh] to binary16 words in groups of G components per
// site, [M][ceil(K/G)][Vh][G], the last group padded with zero words: the FP16
// links (M = 8 parity x direction planes, K = 9, G = 3: one row per group) and
// clover blocks (M = 2, K = 18, G = 4) of the stencil's wide loads.
__global__ void k_regroup16(const double2* __restrict__ src, uint32_t* __restrict__ dst, int M, int K, int G, int Vh) {
    const int NQ = (K + G - 1) / G;
    const long n = (long)M * NQ * Vh * G;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int w = (int)(i % G);
    const long r = i / G;
    const int site = (int)(r % Vh);
    const long mq = r / Vh;
    const int q = (int)(mq % NQ), m = (int)(mq / NQ);
    const int k = q * G + w;
    uint32_t out = 0;
    if (k < K) {
        const double2 v = src[((long)m * K + k) * Vh + site];
        out = f_to_h((float)v.x) | (f_to_h((float)v.y) << 16);
    }
    dst[i] = out;
}

hipError_t launch_regroup16(const double2* src, void* dst, int M, int K, int G, int Vh, hipStream_t s) {
    const long n = (long)M * ((K + G - 1) / G) * Vh * G;
    hipLaunchKernelGGL(k_regroup16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, (uint32_t*)dst, M, K, G, Vh);
    return hipGetLastError();
}

// ---------------------------------------------------------------- canonical <-> even-odd

// Layout conversion between the canonical order (per right-hand side: sites in
// lexicographic order, 12 complex components each) and the even-odd solver order
// (per right-hand side and parity: 12 component planes of Vh sites).  A block moves
// 256 consecutive canonical sites of one right-hand side through LDS, so that both
// sides are read and written in long contiguous runs: the canonical side as one
// 48 KB span, the even-odd side as runs of consecutive checkerboard indices within
// a component plane (the sites s and s+1 of a pair share s/2 and have opposite
// parities; X is even).
constexpr int LAYOUT_BS = 256;

template <bool TO_EO>
__global__ void __launch_bounds__(LAYOUT_BS) k_layout(const double2* __restrict__ src, double2* __restrict__ dst, Geo g, int g5) {
    __shared__ double2 buf[LAYOUT_BS * 12];
    const long V = 2L * g.Vh;
    const int r = blockIdx.y;
    const long s0 = (long)blockIdx.x * LAYOUT_BS;
    const int ns = (int)(V - s0 < LAYOUT_BS ? V - s0 : LAYOUT_BS);  // sites in this block (even)
    const size_t eo0 = (size_t)r * 2 * 12 * g.Vh;
    // pair q = site pair (s0 + 2q, s0 + 2q + 1), half h selects one of them
    const int q = (int)threadIdx.x & (LAYOUT_BS / 2 - 1), h = (int)threadIdx.x / (LAYOUT_BS / 2);
    const long sp = s0 + 2 * q + h;
    int par = 0;
    if (2 * q + h < ns) {
        const Coord c = coord_of(g, sp);
        par = (c.c[0] + c.c[1] + c.c[2] + c.c[3]) & 1;
    }
    const long cb = sp >> 1;
    if (TO_EO) {
        const double2* can = src + ((size_t)r * V + s0) * 12;
        for (int e = threadIdx.x; e < ns * 12; e += LAYOUT_BS) buf[e] = can[e];
        __syncthreads();
        if (2 * q + h < ns) {
            double2* o = dst + eo0 + (size_t)par * 12 * g.Vh + cb;
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                double2 v = buf[(2 * q + h) * 12 + k];
                if (g5 && k >= 6) v = make_double2(-v.x, -v.y);  // g5 = diag(1,1,-1,-1) in spin
                o[(size_t)k * g.Vh] = v;
            }
        }
    } else {
        if (2 * q + h < ns) {
            const double2* in = src + eo0 + (size_t)par * 12 * g.Vh + cb;
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                double2 v = in[(size_t)k * g.Vh];
                if (g5 && k >= 6) v = make_double2(-v.x, -v.y);
                buf[(2 * q + h) * 12 + k] = v;
            }
        }
        __syncthreads();
        double2* o = dst + ((size_t)r * V + s0) * 12;
        for (int e = threadIdx.x; e < ns * 12; e += LAYOUT_BS) o[e] = buf[e];
    }
}

hipError_t launch_canon_to_eo(const double2* can, double2* eo, const Geo& g, int nrhs, hipStream_t s, int g5) {
    if (nrhs <= 0) return hipSuccess;
    long V = 2L * g.Vh;
    for (int r0 = 0; r0 < nrhs; r0 += 65535) {
        int n = nrhs - r0 < 65535 ? nrhs - r0 : 65535;
        hipLaunchKernelGGL(k_layout<true>, dim3((unsigned)((V + LAYOUT_BS - 1) / LAYOUT_BS), n), dim3(LAYOUT_BS), 0, s,
                           can + (size_t)r0 * V * 12, eo + (size_t)r0 * V * 12, g, g5);
    }
    return hipGetLastError();
}

hipError_t launch_eo_to_canon(const double2* eo, double2* can, const Geo& g, int nrhs, hipStream_t s, int g5) {
    if (nrhs <= 0) return hipSuccess;
    long V = 2L * g.Vh;
    for (int r0 = 0; r0 < nrhs; r0 += 65535) {
        int n = nrhs - r0 < 65535 ? nrhs - r0 : 65535;
        hipLaunchKernelGGL(k_layout<false>, dim3((unsigned)((V + LAYOUT_BS - 1) / LAYOUT_BS), n), dim3(LAYOUT_BS), 0, s,
                           eo + (size_t)r0 * V * 12, can + (size_t)r0 * V * 12, g, g5);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- vector kernels

template <int P> __device__ __forceinline__ bool vec_locate(const VecJob<P>* jobs, int njob, const VecJob<P>*& J, int& r, int& cb, int& sb) {
    int bid = blockIdx.x;
    int jb = 0;
    while (jb + 1 < njob && bid >= jobs[jb + 1].blk0) ++jb;
    J = &jobs[jb];
    int lb = bid - J->blk0;
    r = lb / J->nsb;
    sb = lb - r * J->nsb;
    cb = sb * VEC_BS + (int)threadIdx.x;
    return true;
}

template <int BS> __device__ __forceinline__ void write_partial(double v, double* part, long idx) {
    __shared__ double lds[BS / 64];
    double s = block_sum<BS>(v, lds);
    if (threadIdx.x == 0) part[idx] = s;
}

// c = C a (FP64, clover blocks of one parity)
__global__ void __launch_bounds__(VEC_BS) k_clover_apply64(const VecJob<P64>* jobs, int njob) {
    const VecJob<P64>* J; int r, cb, sb;
    vec_locate(jobs, njob, J, r, cb, sb);
    if (cb >= J->Vh) return;
    double x[24], y[24];
    if (!tsup_any(J->tsup, J->T, r, J->vt > 0 ? cb / J->vt : 0, J->tdil)) {  // a is zero here
        for (int i = 0; i < 24; ++i) y[i] = 0.0;
        store_spinor<P64, double>(J->c, J->Vh, r, cb, y);
        return;
    }
    load_spinor<P64, double>(J->a, J->Vh, r, cb, x);
    for (int blk = 0; blk < 2; ++blk) {
        double c[36];
        load_clover_block<P64, double>(J->C, J->Vh, blk, cb, c);
        herm6<double>(c, &x[blk * 12], &y[blk * 12]);
    }
    store_spinor<P64, double>(J->c, J->Vh, r, cb, y);
}

__global__ void __launch_bounds__(256) k_tdist(const int* flags, int* dist, int nrhs, int T) {
    const int i = blockIdx.x * 256 + (int)threadIdx.x;
    if (i >= nrhs * T) return;
    const int r = i / T, t = i - r * T;
    int best = 1 << 28;
    for (int u = 0; u < T; ++u)
        if (flags[(size_t)r * T + u]) {
            const int d = t > u ? t - u : u - t;
            best = min(best, min(d, T - d));
        }
    dist[i] = best;
}

hipError_t launch_tdist(const int* flags, int* dist, int nrhs, int T, hipStream_t s) {
    if (nrhs * T <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tdist, dim3((unsigned)((nrhs * T + 255) / 256)), dim3(256), 0, s, flags, dist, nrhs, T);
    return hipGetLastError();
}

hipError_t launch_clover_apply64(const VecJob<P64>* j, int njob, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_clover_apply64, dim3(nblocks), dim3(VEC_BS), 0, s, j, njob);
    return hipGetLastError();
}

// a = b = P(src / |src|), c = 0 (inner CG start on the unit-norm Schur source:
// r = p = bhat/|bhat|, x = 0); s[r] = |src|^2; part = |a|^2 as stored
template <int P> __global__ void __launch_bounds__(VEC_BS) k_conv_from64(const VecJob<P>* jobs, int njob, const VecJob<P64>* j64) {
    const VecJob<P>* J; int r, cb, sb;
    vec_locate(jobs, njob, J, r, cb, sb);
    const VecJob<P64>* S = &j64[J - jobs];
    double nrm = 0;
    if (J->active && !J->active[r]) {  // right-hand side not iterated this pass (uniform per block)
        if (threadIdx.x == 0) J->part[(long)r * J->pstride + sb] = 0.0;
        return;
    }
    if (cb < J->Vh) {
        double x[24];
        if (tsup_any(S->tsup, S->T, r, S->vt > 0 ? cb / S->vt : 0, S->tdil)) load_spinor<P64, double>(S->a, J->Vh, r, cb, x);
        else for (int i = 0; i < 24; ++i) x[i] = 0.0;  // the source is zero here
        double n2 = J->s[r];
        double sc = n2 > 0 ? 1.0 / sqrt(n2) : 0.0;
        typename PT<P>::R y[24], z[24];
        for (int i = 0; i < 24; ++i) { y[i] = (typename PT<P>::R)(x[i] * sc); z[i] = 0; nrm += (double)y[i] * (double)y[i]; }
        store_spinor<P, typename PT<P>::R>(J->a, J->Vh, r, cb, y);
        store_spinor<P, typename PT<P>::R>(J->b, J->Vh, r, cb, y);
        store_spinor<P, typename PT<P>::R>(J->c, J->Vh, r, cb, z);
    }
    write_partial<VEC_BS>(nrm, J->part, (long)r * J->pstride + sb);
}

template <int P> hipError_t launch_conv_from64(const VecJob<P>* j, int njob, int nblocks, const VecJob<P64>* j64, hipStream_t s) {
    hipLaunchKernelGGL(k_conv_from64<P>, dim3(nblocks), dim3(VEC_BS), 0, s, j, njob, j64);
    return hipGetLastError();
}

// e64 = |bhat| e (back to the scale of the Schur source, FP64), x64 += e64; a right-hand
// side not iterated this pass gets e64 = 0 and keeps x64
template <int P> __global__ void __launch_bounds__(VEC_BS) k_accum_to64(const VecJob<P>* jobs, const VecJob<P64>* j64, int njob) {
    const VecJob<P>* J; int r, cb, sb;
    vec_locate(jobs, njob, J, r, cb, sb);
    if (cb >= J->Vh) return;
    const VecJob<P64>* S = &j64[J - jobs];
    // S->a receives the FP64 copy of the correction; a null view skips it (the FP16
    // solves' reconstruction reads the FP16 field itself, through load_spinor16_f64)
    const bool keep = S->a.v != nullptr;
    if (J->active && !J->active[r]) {
        double z[24];
        for (int i = 0; i < 24; ++i) z[i] = 0.0;
        if (keep) store_spinor<P64, double>(S->a, J->Vh, r, cb, z);
        return;
    }
    double sc = sqrt(J->s[r]);
    double ed[24], x[24];
    if constexpr (P == P16) {
        load_spinor16_f64(J->a, J->Vh, r, cb, sc, ed);
    } else {
        typename PT<P>::R e[24];
        load_spinor<P, typename PT<P>::R>(J->a, J->Vh, r, cb, e);
        for (int i = 0; i < 24; ++i) ed[i] = (double)e[i] * sc;
    }
    load_spinor<P64, double>(S->b, J->Vh, r, cb, x);
    for (int i = 0; i < 24; ++i) x[i] += ed[i];
    if (keep) store_spinor<P64, double>(S->a, J->Vh, r, cb, ed);
    store_spinor<P64, double>(S->b, J->Vh, r, cb, x);
}

template <int P> hipError_t launch_accum_to64(const VecJob<P>* j, const VecJob<P64>* j64, int njob, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_accum_to64<P>, dim3(nblocks), dim3(VEC_BS), 0, s, j, j64, njob);
    return hipGetLastError();
}

// b = a + s[r] * b for active right-hand sides
template <int P> __global__ void __launch_bounds__(VEC_BS) k_xpay(const VecJob<P>* jobs, int njob) {
    const VecJob<P>* J; int r, cb, sb;
    vec_locate(jobs, njob, J, r, cb, sb);
    if (cb >= J->Vh) return;
    if (J->active && !J->active[r]) return;
    using R = typename PT<P>::R;
    R a[24], b[24];
    const R be = (R)J->s[r];
    load_spinor<P, R>(J->a, J->Vh, r, cb, a);
    load_spinor<P, R>(J->b, J->Vh, r, cb, b);
    for (int i = 0; i < 24; ++i) b[i] = a[i] + be * b[i];
    store_spinor<P, R>(J->b, J->Vh, r, cb, b);
}

template <int P> hipError_t launch_xpay(const VecJob<P>* j, int njob, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_xpay<P>, dim3(nblocks), dim3(VEC_BS), 0, s, j, njob);
    return hipGetLastError();
}

template <int P> __global__ void __launch_bounds__(VEC_BS) k_norm(const VecJob<P>* jobs, int njob) {
    const VecJob<P>* J; int r, cb, sb;
    vec_locate(jobs, njob, J, r, cb, sb);
    double nrm = 0;
    const int t = (cb < J->Vh && J->vt > 0) ? cb / J->vt : -1;
    bool nz = false;
    if (cb < J->Vh && tsup_any(J->tsup, J->T, r, t, J->tdil)) {
        typename PT<P>::R a[24];
        load_spinor<P, typename PT<P>::R>(J->a, J->Vh, r, cb, a);
        for (int i = 0; i < 24; ++i) {
            nrm += (double)a[i] * (double)a[i];
            nz = nz || a[i] != 0;  // NaN counts as nonzero
        }
    }
    if (J->tsup_out) {
        // record the timeslices where a is nonzero: one atomic per run of lanes of the
        // wave with a nonzero site on the same timeslice
        const int lane = (int)threadIdx.x & 63;
        const int tu = __shfl_up(t, 1, 64);
        const int nzu = __shfl_up(nz ? 1 : 0, 1, 64);
        if (nz && t >= 0 && (lane == 0 || tu != t || !nzu)) atomicOr(&J->tsup_out[(size_t)r * J->T + t], 1);
    }
    write_partial<VEC_BS>(nrm, J->part, (long)r * J->pstride + sb);
}

template <int P> hipError_t launch_norm(const VecJob<P>* j, int njob, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_norm<P>, dim3(nblocks), dim3(VEC_BS), 0, s, j, njob);
    return hipGetLastError();
}

// deterministic pseudo-random fill (benchmark inputs): splitmix64 of the element index
template <int P> __global__ void k_fill_random(SF<P> f, int Vh, int nrhs, unsigned seed) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)Vh * nrhs) return;
    int r = (int)(i / Vh);
    int cb = (int)(i - (long)r * Vh);
    typename PT<P>::R v[24];
    for (int k = 0; k < 24; ++k) {
        uint64_t z = (uint64_t)seed * 0x9E3779B97F4A7C15ull + (uint64_t)(i * 24 + k) + 1;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        v[k] = (typename PT<P>::R)((double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5);
    }
    store_spinor<P, typename PT<P>::R>(f, Vh, r, cb, v);
}

template <int P> hipError_t launch_fill_random(SF<P> f, int Vh, int nrhs, unsigned seed, hipStream_t s) {
    long n = (long)Vh * nrhs;
    hipLaunchKernelGGL(k_fill_random<P>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, f, Vh, nrhs, seed);
    return hipGetLastError();
}

// diagnostics: out[0] += non-finite values, out[1] += sites whose largest |component| is
// nonzero but below FLT_MIN, out[2] = min over sites of the nonzero largest |component|
template <int P> __global__ void k_check_field(SF<P> f, int Vh, int nrhs, double* out) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)Vh * nrhs) return;
    int r = (int)(i / Vh);
    int cb = (int)(i - (long)r * Vh);
    typename PT<P>::R v[24];
    load_spinor<P, typename PT<P>::R>(f, Vh, r, cb, v);
    double bad = 0, m = 0;
    for (int k = 0; k < 24; ++k) {
        double x = (double)v[k];
        if (!isfinite(x)) bad += 1;
        else m = fmax(m, fabs(x));
    }
    if (bad > 0) atomicAdd(&out[0], bad);
    if (m > 0 && m < 1.17549435e-38) atomicAdd(&out[1], 1.0);
    if (m > 0) atomicMin((unsigned long long*)&out[2], (unsigned long long)__double_as_longlong(m));
    if (P == P16 && f.nrm[(size_t)r * f.ns + cb] > 0) {
        double nm = f.nrm[(size_t)r * f.ns + cb];
        atomicMin((unsigned long long*)&out[3], (unsigned long long)__double_as_longlong(nm));
    }
    if (P == P16 && f.nrm[(size_t)r * f.ns + cb] != f.nrm[(size_t)r * f.ns + cb]) atomicAdd(&out[0], 1000.0);
}

template <int P> hipError_t launch_check_field(SF<P> f, int Vh, int nrhs, double* out, hipStream_t s) {
    long n = (long)Vh * nrhs;
    hipLaunchKernelGGL(k_check_field<P>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, f, Vh, nrhs, out);
    return hipGetLastError();
}

#define DLMA_INST_VEC(P)                                                                                       \
    template hipError_t launch_conv_from64<P>(const VecJob<P>*, int, int, const VecJob<P64>*, hipStream_t); \
    template hipError_t launch_accum_to64<P>(const VecJob<P>*, const VecJob<P64>*, int, int, hipStream_t); \
    template hipError_t launch_xpay<P>(const VecJob<P>*, int, int, hipStream_t);                           \
    template hipError_t launch_norm<P>(const VecJob<P>*, int, int, hipStream_t);                           \
    template hipError_t launch_fill_random<P>(SF<P>, int, int, unsigned, hipStream_t);          \
    template hipError_t launch_check_field<P>(SF<P>, int, int, double*, hipStream_t);
DLMA_INST_VEC(P64)
DLMA_INST_VEC(P32)
DLMA_INST_VEC(P16)
DLMA_INST_VEC(PB16)

// ---------------------------------------------------------------- reduction finishers

// One block per right-hand side: each thread sums a fixed strided subset of the
// partials, then a fixed tree; the result does not depend on launch timing.
__global__ void __launch_bounds__(256) k_finish(const FinJob* jobs, int njob, int mode) {
    int bid = blockIdx.x;
    int jb = 0;
    while (jb + 1 < njob && bid >= jobs[jb + 1].rhs0) ++jb;
    const FinJob& J = jobs[jb];
    int r = bid - J.rhs0;
    if (r >= J.nrhs) return;
    double s = 0;
    for (int i = threadIdx.x; i < J.npart; i += 256) s += J.part[(size_t)r * J.npart + i];
    __shared__ double lds[4];
    s = block_sum<256>(s, lds);
    if (threadIdx.x != 0) return;
    bool finite = isfinite(s);
    if (mode == FIN_NORM) {
        J.out[r] = s;
    } else if (mode == FIN_INIT) {
        // start of an inner solve: |r|^2 = s; active unless already below target
        J.rr[r] = s;
        J.rr0[r] = s;
        // targets refer to the unit-norm source: the absolute one is divided by |bhat|^2
        double sc2 = J.out[r];
        J.tol2[r] = fmax(J.rel2 * s, sc2 > 0 ? J.abs2[r] / sc2 : 0.0);
        J.iters[r] = 0;
        J.alpha[r] = 0;
        J.beta[r] = 0;
        if (J.active[r]) J.active[r] = (finite && s > J.tol2[r]) ? 1 : 0;
    } else if (mode == FIN_ALPHA) {
        if (J.active[r]) {
            if (finite && s > 0.0) {
                J.alpha[r] = J.rr[r] / s;
            } else {
                J.alpha[r] = 0.0;
                J.active[r] = 0;
            }
        } else {
            J.alpha[r] = 0.0;
        }
    } else {  // FIN_BETA
        if (J.active[r]) {
            J.beta[r] = s / J.rr[r];
            J.rr[r] = s;
            int it = J.iters[r] + 1;
            J.iters[r] = it;
            if (!finite || s <= J.tol2[r] || it >= J.maxit) J.active[r] = 0;
        } else {
            J.beta[r] = 0.0;
        }
    }
}

hipError_t launch_finish(const FinJob* j, int njob, int nblocks, int mode, hipStream_t s) {
    hipLaunchKernelGGL(k_finish, dim3(nblocks), dim3(256), 0, s, j, njob, mode);
    return hipGetLastError();
}


// ---------------------------------------------------------------- measurement

typedef uint32_t cp32x4 __attribute__((ext_vector_type(4)));

// b = a over n 16-byte words: the plain streaming copy that measures the memory
// system's read + write bandwidth.  Four independent 128-bit loads per thread are in
// flight before their stores; both bypass the caches' retention (non-temporal).
__global__ void __launch_bounds__(256) k_stream_copy(const cp32x4* __restrict__ a, cp32x4* __restrict__ b, long n) {
    const long stride = (long)gridDim.x * 256;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += 4 * stride) {
        cp32x4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i + k * stride < n) v[k] = __builtin_nontemporal_load(a + i + k * stride);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i + k * stride < n) __builtin_nontemporal_store(v[k], b + i + k * stride);
    }
}

hipError_t launch_stream_copy(const void* a, void* b, long n16, hipStream_t s) {
    long blocks = (n16 + 1023) / 1024;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, s, (const cp32x4*)a, (cp32x4*)b, n16);
    return hipGetLastError();
}

}  // namespace dlma
