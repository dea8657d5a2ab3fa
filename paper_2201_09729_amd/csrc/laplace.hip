// Spatial covariant Laplacian (paper eq. 1) on a batch of timeslices, the
// kernels of the batched Lanczos eigensolver, and the distillation projector.
//
// Colour vectors are complex128 in the canonical [site3][colour] order of one
// timeslice, site3 = (z*Y + y)*X + x; n = 3 L^3 complex numbers per vector.
// A batch of vectors for nt timeslices is addressed as base + t * tstride.
#include "laplace.h"

namespace dlma {

__device__ __forceinline__ double2 cmul2(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ double2 cconjmul(double2 a, double2 b) {  // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Chebyshev-filter mode of the stencil: out = c2 * (c1 * in - (-lap) in) - prev
struct LapMode {
    int cheb;            // 0: out = -lap in;  1: out = c2 (c1 in + lap in) - prev
    double c1, c2;
    const double2* prev; // timeslice stride tsp, vector stride as in; nullptr = 0
    long tsp;
    const double2* qd;   // one vector per timeslice (stride tsqd): block partials of Re <qd, out>; nullptr = none
    long tsqd;
    double* part;        // [nt][gridDim.x] partials for qd
};

// out = -lap(t) in = 6 in - sum_j [U_j(m,t) in(m+j) + U_j(m-j,t)^dag in(m-j)],  j = x, y, z,
// for nv vectors on each of nt timeslices: vector (tl, kv) at base + tl*tstride + kv*vstride.
// Grid: (site blocks of one timeslice, ceil(nv / VPT), nt).  Each thread takes VPT
// vectors at one site: the six links of the site are loaded once and applied to all
// of them, which halves the load instructions per vector at VPT = 4 (the kernel is
// bound by the texture address path, like the stencils).  The partials of qd are
// for nv = 1 (one vector per timeslice).
template <int VPT>
__global__ void __launch_bounds__(256) k_neg_lap(const double2* __restrict__ U64, Geo g, int t0, const double2* __restrict__ in,
                                                 double2* __restrict__ out, long tstride_in, long tstride_out, long vstride_in,
                                                 long vstride_out, int nv, LapMode md) {
    const int L3 = g.Z * g.Y * g.X;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    const int kv0 = blockIdx.y * VPT, tl = blockIdx.z;
    const int nk = min(VPT, nv - kv0);  // uniform over the block
    double dq = 0.0;
    if (m < L3) {
        const int t = t0 + tl;
        int x = m % g.X, y = (m / g.X) % g.Y, z = m / (g.X * g.Y);
        const double2* v = in + tl * tstride_in + kv0 * vstride_in;
        double2 acc[VPT][3];
#pragma unroll
        for (int i = 0; i < VPT; ++i)
            if (i < nk)
                for (int a = 0; a < 3; ++a) {
                    double2 q = v[i * vstride_in + (long)m * 3 + a];
                    acc[i][a] = make_double2(6.0 * q.x, 6.0 * q.y);
                }
        for (int j = 1; j <= 3; ++j) {
            int xf = x, yf = y, zf = z, xb = x, yb = y, zb = z;
            if (j == 1) { xf = x + 1 == g.X ? 0 : x + 1; xb = x == 0 ? g.X - 1 : x - 1; }
            if (j == 2) { yf = y + 1 == g.Y ? 0 : y + 1; yb = y == 0 ? g.Y - 1 : y - 1; }
            if (j == 3) { zf = z + 1 == g.Z ? 0 : z + 1; zb = z == 0 ? g.Z - 1 : z - 1; }
            int mf = (zf * g.Y + yf) * g.X + xf, mb = (zb * g.Y + yb) * g.X + xb;
            // link U_j at (t, m) and at the backward neighbour (t, m - j)
            int par = (t + z + y + x) & 1, parb = (t + zb + yb + xb) & 1;
            long cb = (((long)t * g.Z + z) * g.Y + y) * g.Xh + (x >> 1);
            long cbb = (((long)t * g.Z + zb) * g.Y + yb) * g.Xh + (xb >> 1);
            const double2* uf = U64 + ((size_t)(par * 4 + j) * 9) * g.Vh + cb;
            const double2* ub = U64 + ((size_t)(parb * 4 + j) * 9) * g.Vh + cbb;
            double2 u[9], w[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) { u[e] = uf[(size_t)e * g.Vh]; w[e] = ub[(size_t)e * g.Vh]; }
#pragma unroll
            for (int i = 0; i < VPT; ++i)
                if (i < nk) {
                    const double2* vi = v + i * vstride_in;
                    double2 vf[3], vb[3];
                    for (int b = 0; b < 3; ++b) { vf[b] = vi[(long)mf * 3 + b]; vb[b] = vi[(long)mb * 3 + b]; }
                    for (int a = 0; a < 3; ++a) {
                        double2 sm = make_double2(0, 0);
                        for (int b = 0; b < 3; ++b) {
                            double2 p = cmul2(u[a * 3 + b], vf[b]);
                            double2 q = cconjmul(w[b * 3 + a], vb[b]);  // (U^dag)_{ab} = conj(U_{ba})
                            sm.x += p.x + q.x;
                            sm.y += p.y + q.y;
                        }
                        acc[i][a].x -= sm.x;
                        acc[i][a].y -= sm.y;
                    }
                }
        }
#pragma unroll
        for (int i = 0; i < VPT; ++i)
            if (i < nk) {
                double2* o = out + tl * tstride_out + (kv0 + i) * vstride_out;
                if (md.cheb) {
                    const double2* pv = md.prev ? md.prev + tl * md.tsp + (kv0 + i) * vstride_in : nullptr;
                    for (int a = 0; a < 3; ++a) {
                        double2 q = v[i * vstride_in + (long)m * 3 + a], pr = pv ? pv[(long)m * 3 + a] : make_double2(0.0, 0.0);
                        acc[i][a] = make_double2(md.c2 * (md.c1 * q.x - acc[i][a].x) - pr.x, md.c2 * (md.c1 * q.y - acc[i][a].y) - pr.y);
                    }
                }
                for (int a = 0; a < 3; ++a) o[(long)m * 3 + a] = acc[i][a];
            }
        if (md.qd) {
            const double2* pq = md.qd + tl * md.tsqd + (long)m * 3;
            for (int a = 0; a < 3; ++a) dq += pq[a].x * acc[0][a].x + pq[a].y * acc[0][a].y;
        }
    }
    if (md.qd) {  // uniform over the grid
        __shared__ double lds[4];
        dq = block_sum<256>(dq, lds);
        if (threadIdx.x == 0) md.part[(long)tl * gridDim.x + blockIdx.x] = dq;
    }
}

// vectors per thread of a launch over nv vectors
constexpr int LAP_VPT = 4;
static hipError_t launch_lap(const double2* U64, const Geo& g, int t0, const double2* in, double2* out, long tsi, long tso,
                             int nt, int nv, long vsi, long vso, const LapMode& md, hipStream_t s);

int lap_site_blocks(const Geo& g) { return (g.Z * g.Y * g.X + 255) / 256; }

hipError_t launch_neg_lap(const double2* U64, const Geo& g, int t0, const double2* in, double2* out, long tsi, long tso,
                          int nt, hipStream_t s, int nv, long vsi, long vso, const double2* qd, double* part) {
    if (nt <= 0 || nv <= 0) return hipSuccess;
    LapMode md = {0, 0.0, 0.0, nullptr, 0L, qd, tsi, part};
    return launch_lap(U64, g, t0, in, out, tsi, tso, nt, nv, vsi, vso, md, s);
}

static hipError_t launch_lap(const double2* U64, const Geo& g, int t0, const double2* in, double2* out, long tsi, long tso,
                             int nt, int nv, long vsi, long vso, const LapMode& md, hipStream_t s) {
    if (nv == 1 || md.qd) {  // partials of qd: one vector per thread
        hipLaunchKernelGGL(k_neg_lap<1>, dim3((unsigned)lap_site_blocks(g), nv, nt), dim3(256), 0, s, U64, g, t0, in, out, tsi,
                           tso, vsi, vso, nv, md);
    } else {
        hipLaunchKernelGGL(k_neg_lap<LAP_VPT>, dim3((unsigned)lap_site_blocks(g), (nv + LAP_VPT - 1) / LAP_VPT, nt), dim3(256),
                           0, s, U64, g, t0, in, out, tsi, tso, vsi, vso, nv, md);
    }
    return hipGetLastError();
}

// out = c2 * (c1 * in - (-lap) in) - prev  (one step of the Chebyshev three-term recurrence)
hipError_t launch_cheb_step(const double2* U64, const Geo& g, int t0, const double2* in, long tsi, const double2* prev, long tsp,
                            double2* out, long tso, int nt, double c1, double c2, hipStream_t s, const double2* qd, long tsqd,
                            double* part) {
    if (nt <= 0) return hipSuccess;
    LapMode md = {1, c1, c2, prev, tsp, qd, tsqd, part};
    return launch_lap(U64, g, t0, in, out, tsi, tso, nt, 1, 0L, 0L, md, s);
}

// Per vector: lambda = Re <y, Ay> (y normalised), then |Ay - lambda y|; one block per vector
__global__ void __launch_bounds__(256) k_rayleigh(const double2* __restrict__ y, const double2* __restrict__ ay, long n,
                                                  double* __restrict__ lam, double* __restrict__ res) {
    __shared__ double lds[4];
    const double2* py = y + (long)blockIdx.x * n;
    const double2* pa = ay + (long)blockIdx.x * n;
    double d = 0, nn = 0;
    for (long e = threadIdx.x; e < n; e += 256) {
        d += py[e].x * pa[e].x + py[e].y * pa[e].y;
        nn += py[e].x * py[e].x + py[e].y * py[e].y;
    }
    d = block_sum<256>(d, lds);
    nn = block_sum<256>(nn, lds);
    __shared__ double l;
    if (threadIdx.x == 0) l = d / nn;
    __syncthreads();
    double r = 0;
    for (long e = threadIdx.x; e < n; e += 256) {
        double rx = pa[e].x - l * py[e].x, ry = pa[e].y - l * py[e].y;
        r += rx * rx + ry * ry;
    }
    r = block_sum<256>(r, lds);
    if (threadIdx.x == 0) {
        lam[blockIdx.x] = l;
        res[blockIdx.x] = sqrt(r / nn);
    }
}

hipError_t launch_rayleigh(const double2* y, const double2* ay, long n, int nvec, double* lam, double* res, hipStream_t s) {
    hipLaunchKernelGGL(k_rayleigh, dim3(nvec), dim3(256), 0, s, y, ay, n, lam, res);
    return hipGetLastError();
}

// ---------------------------------------------------------------- batched reductions

template <int BS> __device__ __forceinline__ double2 block_sum2(double2 v, double* lds) {
    v.x = block_sum<BS>(v.x, lds);
    v.y = block_sum<BS>(v.y, lds);
    return v;
}

// out[t * ostride + i] = <a_{t,i}, b_t> for i < ni (grid: ni x nt); a_{t,i} = a + t*tsa + i*isa
__global__ void __launch_bounds__(256) k_dots(const double2* __restrict__ a, long tsa, long isa, const double2* __restrict__ b,
                                              long tsb, long n, double2* __restrict__ out, int ostride) {
    __shared__ double lds[4];
    int i = blockIdx.x, t = blockIdx.y;
    const double2* pa = a + t * tsa + i * isa;
    const double2* pb = b + t * tsb;
    double2 s = make_double2(0, 0);
    for (long e = threadIdx.x; e < n; e += 256) {
        double2 p = cconjmul(pa[e], pb[e]);
        s.x += p.x;
        s.y += p.y;
    }
    s = block_sum2<256>(s, lds);
    if (threadIdx.x == 0) out[(long)t * ostride + i] = s;
}

hipError_t launch_dots(const double2* a, long tsa, long isa, const double2* b, long tsb, long n, double2* out, int ostride,
                       int ni, int nt, hipStream_t s) {
    if (ni <= 0 || nt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dots, dim3(ni, nt), dim3(256), 0, s, a, tsa, isa, b, tsb, n, out, ostride);
    return hipGetLastError();
}

// beta_t = |w_t|; q_{j+1} = w / beta (beta below 1e-300 leaves q_{j+1} = 0)
__global__ void __launch_bounds__(256) k_norm_t(const double2* __restrict__ w, long tsw, long n, double* __restrict__ out,
                                                int ostride, int j) {
    __shared__ double lds[4];
    int t = blockIdx.x;
    const double2* pw = w + t * tsw;
    double s = 0;
    for (long e = threadIdx.x; e < n; e += 256) s += pw[e].x * pw[e].x + pw[e].y * pw[e].y;
    s = block_sum<256>(s, lds);
    if (threadIdx.x == 0) out[(long)t * ostride + j] = sqrt(s);
}

__global__ void k_scale_into(const double2* __restrict__ w, long tsw, double2* __restrict__ q, long tsq, long n,
                             const double* __restrict__ nrm, int ostride, int j) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    int t = blockIdx.y;
    if (e >= n) return;
    double b = nrm[(long)t * ostride + j];
    double inv = b > 1e-300 ? 1.0 / b : 0.0;
    double2 v = w[t * tsw + e];
    q[t * tsq + e] = make_double2(v.x * inv, v.y * inv);
}

hipError_t launch_normalize_into(const double2* w, long tsw, double2* q, long tsq, long n, double* nrm, int ostride, int j, int nt,
                                 hipStream_t s) {
    hipLaunchKernelGGL(k_norm_t, dim3(nt), dim3(256), 0, s, w, tsw, n, nrm, ostride, j);
    hipLaunchKernelGGL(k_scale_into, dim3((unsigned)((n + 255) / 256), nt), dim3(256), 0, s, w, tsw, q, tsq, n, nrm, ostride, j);
    return hipGetLastError();
}

// ---------------------------------------------------------------- Lanczos step, split reductions
//
// A Lanczos step on one timeslice reduces over 3 L^3 elements several times; one
// block per reduction leaves most of the chip idle and waits on a long serial loop.
// Here every reduction is split over blocks that write partial sums, and the
// kernel that consumes the result adds the partials in a fixed order (the same on
// every thread, so the result is deterministic).

// alpha_t = sum of the block partials of Re <q_j, w> written by the stencil that
// produced w; w -= alpha_t q_j + beta_{j-1} q_{j-1}
__global__ void k_lanczos_three_p(const double2* __restrict__ qj, const double2* __restrict__ qjm, long tsq,
                                  double2* __restrict__ w, long tsw, long n, const double* __restrict__ apart, int nap,
                                  double* __restrict__ alpha, const double* __restrict__ beta, int astride, int j, int prev) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    int t = blockIdx.y;
    double a = 0.0;
    for (int b = 0; b < nap; ++b) a += apart[(long)t * nap + b];
    if (blockIdx.x == 0 && threadIdx.x == 0) alpha[(long)t * astride + j] = a;
    if (e >= n) return;
    double2 v = w[t * tsw + e];
    double2 c = qj[t * tsq + e];
    v.x -= a * c.x;
    v.y -= a * c.y;
    if (prev) {
        double b = beta[(long)t * astride + j - 1];
        double2 d = qjm[t * tsq + e];
        v.x -= b * d.x;
        v.y -= b * d.y;
    }
    w[t * tsw + e] = v;
}

hipError_t launch_lanczos_three_p(const double2* q, long tsq, long isq, double2* w, long tsw, long n, const double* apart, int nap,
                                  double* alpha, double* beta, int astride, int j, int nt, hipStream_t s, bool prev) {
    const double2* qjm = j > 0 ? q + (long)(j - 1) * isq : q;
    hipLaunchKernelGGL(k_lanczos_three_p, dim3((unsigned)((n + 255) / 256), nt), dim3(256), 0, s, q + (long)j * isq, qjm, tsq, w,
                       tsw, n, apart, nap, alpha, beta, astride, j, (prev && j > 0) ? 1 : 0);
    return hipGetLastError();
}

// Partial dots hp[(t * GS_NCH + ch) * hstride + i] = <a_{t,i}, b_t> over chunk ch of the elements
__global__ void __launch_bounds__(256) k_gs_dots(const double2* __restrict__ a, long tsa, long isa, const double2* __restrict__ b,
                                                 long tsb, long n, double2* __restrict__ hp, int hstride) {
    __shared__ double lds[4];
    const int i = blockIdx.x, ch = blockIdx.y, t = blockIdx.z;
    const long clen = (n + GS_NCH - 1) / GS_NCH;
    const long e0 = ch * clen, e1 = e0 + clen < n ? e0 + clen : n;
    const double2* pa = a + t * tsa + i * isa;
    const double2* pb = b + t * tsb;
    double2 s = make_double2(0, 0);
    for (long e = e0 + threadIdx.x; e < e1; e += 256) {
        double2 p = cconjmul(pa[e], pb[e]);
        s.x += p.x;
        s.y += p.y;
    }
    s = block_sum2<256>(s, lds);
    if (threadIdx.x == 0) hp[((long)t * GS_NCH + ch) * hstride + i] = s;
}

hipError_t launch_gs_dots(const double2* a, long tsa, long isa, const double2* b, long tsb, long n, double2* hp, int hstride, int ni,
                          int nt, hipStream_t s) {
    if (ni <= 0 || nt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gs_dots, dim3(ni, GS_NCH, nt), dim3(256), 0, s, a, tsa, isa, b, tsb, n, hp, hstride);
    return hipGetLastError();
}

// w_t -= sum_{i < ni} q_{t,i} h_{t,i} with h the sum of the GS_NCH partials (added into LDS
// tile by tile); with npart, also the block partials of |w_t|^2 after the update
__global__ void __launch_bounds__(256) k_gs_sub(const double2* __restrict__ q, long tsq, long isq, const double2* __restrict__ hp,
                                                int hstride, int ni, double2* __restrict__ w, long tsw, long n,
                                                double* __restrict__ npart) {
    constexpr int TILE = 1024;
    __shared__ double2 h[TILE];
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int t = blockIdx.y;
    const double2* pq = q + t * tsq + e;
    double2 s = make_double2(0, 0);
    for (int i0 = 0; i0 < ni; i0 += TILE) {
        const int nk = ni - i0 < TILE ? ni - i0 : TILE;
        __syncthreads();
        for (int k = threadIdx.x; k < nk; k += 256) {
            double2 v = make_double2(0, 0);
            for (int ch = 0; ch < GS_NCH; ++ch) {
                double2 p = hp[((long)t * GS_NCH + ch) * hstride + i0 + k];
                v.x += p.x;
                v.y += p.y;
            }
            h[k] = v;
        }
        __syncthreads();
        if (e < n)
            for (int k = 0; k < nk; ++k) {
                double2 c = cmul2(pq[(long)(i0 + k) * isq], h[k]);
                s.x += c.x;
                s.y += c.y;
            }
    }
    double nn = 0.0;
    if (e < n) {
        double2* pw = w + t * tsw + e;
        double2 v = *pw;
        v.x -= s.x;
        v.y -= s.y;
        *pw = v;
        nn = v.x * v.x + v.y * v.y;
    }
    if (npart) {  // uniform over the grid
        __shared__ double lds[4];
        nn = block_sum<256>(nn, lds);
        if (threadIdx.x == 0) npart[(long)t * gridDim.x + blockIdx.x] = nn;
    }
}

int gs_sub_blocks(long n) { return (int)((n + 255) / 256); }

hipError_t launch_gs_sub(const double2* q, long tsq, long isq, const double2* hp, int hstride, int ni, double2* w, long tsw, long n,
                         int nt, double* npart, hipStream_t s) {
    if (nt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gs_sub, dim3((unsigned)gs_sub_blocks(n), nt), dim3(256), 0, s, q, tsq, isq, hp, hstride, ni, w, tsw, n,
                       npart);
    return hipGetLastError();
}

// beta_t = sqrt(sum of the nnp block partials of |w_t|^2); q_{j+1} = w / beta
// (beta below 1e-300 leaves q_{j+1} = 0)
__global__ void k_scale_p(const double2* __restrict__ w, long tsw, double2* __restrict__ q, long tsq, long n,
                          const double* __restrict__ npart, int nnp, double* __restrict__ nrm, int ostride, int j) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    int t = blockIdx.y;
    double s = 0.0;
    for (int b = 0; b < nnp; ++b) s += npart[(long)t * nnp + b];
    const double bt = sqrt(s);
    if (blockIdx.x == 0 && threadIdx.x == 0) nrm[(long)t * ostride + j] = bt;
    if (e >= n) return;
    double inv = bt > 1e-300 ? 1.0 / bt : 0.0;
    double2 v = w[t * tsw + e];
    q[t * tsq + e] = make_double2(v.x * inv, v.y * inv);
}

hipError_t launch_scale_p(const double2* w, long tsw, double2* q, long tsq, long n, const double* npart, double* nrm, int ostride,
                          int j, int nt, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_p, dim3((unsigned)gs_sub_blocks(n), nt), dim3(256), 0, s, w, tsw, q, tsq, n, npart,
                       gs_sub_blocks(n), nrm, ostride, j);
    return hipGetLastError();
}

// Ritz vectors: y_{t,k} = sum_{i < m} q_{t,i} S[t][i][k], S row-major [m][nev] per t
__global__ void k_ritz(const double2* __restrict__ q, long tsq, long isq, const double* __restrict__ S, int m, int nev,
                       double2* __restrict__ y, long tsy, long n) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    int t = blockIdx.z;
    int k0 = blockIdx.y * 4;
    if (e >= n) return;
    const double* St = S + (long)t * m * nev;
    double2 acc[4] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
    const double2* pq = q + t * tsq + e;
    for (int i = 0; i < m; ++i) {
        double2 v = pq[(long)i * isq];
        for (int kk = 0; kk < 4; ++kk) {
            if (k0 + kk < nev) {
                double c = St[(long)i * nev + k0 + kk];
                acc[kk].x += c * v.x;
                acc[kk].y += c * v.y;
            }
        }
    }
    for (int kk = 0; kk < 4; ++kk)
        if (k0 + kk < nev) y[t * tsy + (long)(k0 + kk) * n + e] = acc[kk];
}

hipError_t launch_ritz(const double2* q, long tsq, long isq, const double* S, int m, int nev, double2* y, long tsy, long n, int nt,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_ritz, dim3((unsigned)((n + 255) / 256), (nev + 3) / 4, nt), dim3(256), 0, s, q, tsq, isq, S, m, nev, y,
                       tsy, n);
    return hipGetLastError();
}

// Phase convention per vector: the component of largest modulus (lowest index among
// those within 1e-10 of the maximum) becomes real and positive.  One block per vector.
__global__ void __launch_bounds__(256) k_phase_fix(double2* __restrict__ y, long n) {
    __shared__ double red[256];
    __shared__ long ired[256];
    double2* v = y + (long)blockIdx.x * n;
    double mx = 0;
    for (long e = threadIdx.x; e < n; e += 256) mx = fmax(mx, hypot(v[e].x, v[e].y));
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
    }
    double thr = red[0] - 1e-10;
    __syncthreads();
    long first = n;
    for (long e = threadIdx.x; e < n; e += 256)
        if (hypot(v[e].x, v[e].y) >= thr) { first = e; break; }
    ired[threadIdx.x] = first;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) ired[threadIdx.x] = min(ired[threadIdx.x], ired[threadIdx.x + st]);
        __syncthreads();
    }
    long i0 = ired[0];
    if (i0 >= n) return;
    double2 p = v[i0];
    double a = hypot(p.x, p.y);
    if (!(a > 0)) return;
    double2 ph = make_double2(p.x / a, -p.y / a);  // conj(p)/|p|
    __syncthreads();
    for (long e = threadIdx.x; e < n; e += 256) v[e] = cmul2(v[e], ph);
}

hipError_t launch_phase_fix(double2* y, long n, int nvec, hipStream_t s) {
    hipLaunchKernelGGL(k_phase_fix, dim3(nvec), dim3(256), 0, s, y, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------- block eigensolver
//
// Chebyshev-filtered subspace iteration keeps a block of kb vectors per timeslice,
// stored [t][k][n] (vector k of timeslice t at base + (t*kb + k)*n).

// One Chebyshev step on every vector of the block: out = c2 (c1 in - (-lap) in) - prev
hipError_t launch_cheb_block(const double2* U64, const Geo& g, int t0, const double2* in, const double2* prev, double2* out,
                             int nt, int kb, double c1, double c2, hipStream_t s) {
    if (nt <= 0 || kb <= 0) return hipSuccess;
    const long n = 3L * g.Z * g.Y * g.X;
    LapMode md = {1, c1, c2, prev, (long)kb * n, nullptr, 0L, nullptr};
    return launch_lap(U64, g, t0, in, out, (long)kb * n, (long)kb * n, nt, kb, n, n, md, s);
}

// Gram partials: part[t][c][i][j] = sum over rows of chunk c of conj(A_i[e]) B_j[e], i, j < kb.
// Rows are staged through LDS in tiles; each thread owns the (i, j) pairs
// i = ty + 16a, j = tx + 16b (a, b < 4), so kb <= 64.
constexpr int GRAM_ROWS = 16;
__global__ void __launch_bounds__(256) k_block_gram(const double2* __restrict__ A, const double2* __restrict__ B, long n, int kb,
                                                    long chunk, double2* __restrict__ part) {
    __shared__ double2 ta[GRAM_ROWS][64], tb[GRAM_ROWS][64];
    const int c = blockIdx.x, t = blockIdx.y, nc = gridDim.x;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const double2* At = A + (size_t)t * kb * n;
    const double2* Bt = B + (size_t)t * kb * n;
    const long e0 = (long)c * chunk, e1 = e0 + chunk < n ? e0 + chunk : n;
    double2 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0, 0);
    for (long r0 = e0; r0 < e1; r0 += GRAM_ROWS) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < GRAM_ROWS * 64; idx += 256) {
            const int rr = idx / 64, k = idx % 64;
            const long e = r0 + rr;
            const bool ok = e < e1 && k < kb;
            ta[rr][k] = ok ? At[(size_t)k * n + e] : make_double2(0, 0);
            tb[rr][k] = ok ? Bt[(size_t)k * n + e] : make_double2(0, 0);
        }
        __syncthreads();
        for (int rr = 0; rr < GRAM_ROWS; ++rr) {
            double2 av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = ta[rr][ty + 16 * a];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = tb[rr][tx + 16 * b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const double2 p = cconjmul(av[a], bv[b]);
                    acc[a][b].x += p.x;
                    acc[a][b].y += p.y;
                }
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ty + 16 * a, j = tx + 16 * b;
            if (i < kb && j < kb) part[(((size_t)t * nc + c) * kb + i) * kb + j] = acc[a][b];
        }
}

// G[t][i][j] = sum of the chunk partials in chunk order
__global__ void k_block_gram_sum(const double2* __restrict__ part, int nc, int kb, int nt, double2* __restrict__ G) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)nt * kb * kb) return;
    const int t = (int)(idx / ((long)kb * kb));
    const int ij = (int)(idx - (long)t * kb * kb);
    double2 s = make_double2(0, 0);
    for (int c = 0; c < nc; ++c) {
        const double2 p = part[((size_t)t * nc + c) * kb * kb + ij];
        s.x += p.x;
        s.y += p.y;
    }
    G[idx] = s;
}

int block_gram_chunks(long n, int nt) {
    long want = (256 + nt - 1) / nt;  // enough blocks to fill the chip, few partials to add
    long maxc = (n + GRAM_ROWS - 1) / GRAM_ROWS;
    return (int)std::max(1L, std::min(want, maxc));
}

hipError_t launch_block_gram(const double2* A, const double2* B, long n, int kb, int nt, double2* part, double2* G,
                             hipStream_t s) {
    if (kb > 64) return hipErrorInvalidValue;
    const int nc = block_gram_chunks(n, nt);
    long chunk = (n + nc - 1) / nc;
    chunk = (chunk + GRAM_ROWS - 1) / GRAM_ROWS * GRAM_ROWS;
    hipLaunchKernelGGL(k_block_gram, dim3(nc, nt), dim3(256), 0, s, A, B, n, kb, chunk, part);
    const long tot = (long)nt * kb * kb;
    hipLaunchKernelGGL(k_block_gram_sum, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, part, nc, kb, nt, G);
    return hipGetLastError();
}

// Y_j = sum_i X_i Z[t][i][j] for j < kout (Z complex, row-major kb x kout per timeslice);
// grid (row blocks, nt, output groups of 8)
__global__ void __launch_bounds__(256) k_block_update(const double2* __restrict__ X, const double2* __restrict__ Z, long n, int kb,
                                                      int kout, double2* __restrict__ Y, long ytstride) {
    __shared__ double2 zs[64 * 8];
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int t = blockIdx.y, j0 = blockIdx.z * 8;
    const double2* Zt = Z + (size_t)t * kb * kout;
    for (int idx = threadIdx.x; idx < kb * 8; idx += 256) {
        const int i = idx / 8, jj = idx % 8;
        zs[idx] = j0 + jj < kout ? Zt[(size_t)i * kout + j0 + jj] : make_double2(0, 0);
    }
    __syncthreads();
    if (e >= n) return;
    double2 acc[8];
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) acc[jj] = make_double2(0, 0);
    const double2* Xt = X + (size_t)t * kb * n + e;
    for (int i = 0; i < kb; ++i) {
        const double2 x = Xt[(size_t)i * n];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            const double2 p = cmul2(x, zs[i * 8 + jj]);
            acc[jj].x += p.x;
            acc[jj].y += p.y;
        }
    }
    double2* Yt = Y + (size_t)t * ytstride + e;
#pragma unroll
    for (int jj = 0; jj < 8; ++jj)
        if (j0 + jj < kout) Yt[(size_t)(j0 + jj) * n] = acc[jj];
}

hipError_t launch_block_update(const double2* X, const double2* Z, long n, int kb, int kout, int nt, double2* Y, long ytstride,
                               hipStream_t s) {
    if (kb > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_block_update, dim3((unsigned)((n + 255) / 256), nt, (kout + 7) / 8), dim3(256), 0, s, X, Z, n, kb, kout,
                       Y, ytstride);
    return hipGetLastError();
}

// Seeded complex uniform entries in (-1/2, 1/2): splitmix64 of the element index
__global__ void k_block_random(double2* __restrict__ V, long count, unsigned seed) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    double v[2];
    for (int k = 0; k < 2; ++k) {
        uint64_t z = (uint64_t)seed * 0x9E3779B97F4A7C15ull + (uint64_t)(2 * i + k) + 1;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        v[k] = (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    }
    V[i] = make_double2(v[0], v[1]);
}

hipError_t launch_block_random(double2* V, long count, unsigned seed, hipStream_t s) {
    hipLaunchKernelGGL(k_block_random, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, V, count, seed);
    return hipGetLastError();
}

// ---------------------------------------------------------------- projector

// c[r][k][s] = sum_{m,col} conj(V[k][m][col]) in_r(t, m, s, col); one block per (k, r)
__global__ void __launch_bounds__(256) k_proj_coef(const double2* __restrict__ Vt, const double2* __restrict__ in, long L3,
                                                   long tofs, long fstride, int nev, double2* __restrict__ c) {
    __shared__ double lds[4];
    int k = blockIdx.x, r = blockIdx.y;
    const double2* v = Vt + (long)k * L3 * 3;
    const double2* f = in + (long)r * fstride + tofs;
    double2 acc[4] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
    for (long m = threadIdx.x; m < L3; m += 256) {
        for (int col = 0; col < 3; ++col) {
            double2 a = v[m * 3 + col];
            for (int sp = 0; sp < 4; ++sp) {
                double2 p = cconjmul(a, f[(m * 4 + sp) * 3 + col]);
                acc[sp].x += p.x;
                acc[sp].y += p.y;
            }
        }
    }
    for (int sp = 0; sp < 4; ++sp) {
        double2 s = block_sum2<256>(acc[sp], lds);
        if (threadIdx.x == 0) c[((long)r * nev + k) * 4 + sp] = s;
    }
}

// out_r = box(t) in_r (mode 0) or (1 - box(t)) in_r (mode 1) on timeslice t, 0 elsewhere
__global__ void k_proj_apply(const double2* __restrict__ Vt, const double2* in, double2* out, long L3, long V, int t, int nev,
                             const double2* __restrict__ c, int mode) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;  // over V sites x 4 spins
    int r = blockIdx.y;
    if (i >= V * 4) return;
    long site = i >> 2;
    int sp = (int)(i & 3);
    long base = ((long)r * V * 4 + i) * 3;
    long tt = site / L3;
    if (tt != t) {
        for (int col = 0; col < 3; ++col) out[base + col] = make_double2(0, 0);
        return;
    }
    long m = site - (long)t * L3;
    double2 acc[3] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
    const double2* cr = c + (long)r * nev * 4;
    for (int k = 0; k < nev; ++k) {
        double2 ck = cr[k * 4 + sp];
        for (int col = 0; col < 3; ++col) {
            double2 p = cmul2(Vt[((long)k * L3 + m) * 3 + col], ck);
            acc[col].x += p.x;
            acc[col].y += p.y;
        }
    }
    for (int col = 0; col < 3; ++col) {
        double2 o = acc[col];
        if (mode == 1) {
            double2 x = in[base + col];
            o = make_double2(x.x - o.x, x.y - o.y);
        }
        out[base + col] = o;
    }
}

hipError_t launch_project(const double2* Vt, const double2* in, double2* out, const Geo& g, int t, int nev, int nrhs, int mode,
                          double2* coef, hipStream_t s) {
    long L3 = (long)g.Z * g.Y * g.X;
    long V = 2L * g.Vh;
    for (int r0 = 0; r0 < nrhs; r0 += 65535) {
        int nr = nrhs - r0 < 65535 ? nrhs - r0 : 65535;
        const double2* inr = in + (long)r0 * V * 12;
        double2* outr = out + (long)r0 * V * 12;
        if (nev > 0)  // no modes: box(t) = 0 and the apply kernel reads no coefficient
            hipLaunchKernelGGL(k_proj_coef, dim3(nev, nr), dim3(256), 0, s, Vt, inr, L3, (long)t * L3 * 12, V * 12, nev, coef);
        hipLaunchKernelGGL(k_proj_apply, dim3((unsigned)((V * 4 + 255) / 256), nr), dim3(256), 0, s, Vt, inr, outr, L3, V, t, nev,
                           coef, mode);
    }
    return hipGetLastError();
}

}  // namespace dlma
