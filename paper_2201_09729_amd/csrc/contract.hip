// Timeslice contractions behind the correlators (paper eq. 2-4):
//   tproj:     P[f][t][k][s] = sum_{m,c} conj(V_k(t)(m,c)) phi_f(t,m,s,c)
//              (projections of solutions on the Laplacian modes; for the
//              distillation solutions this is the perambulator)
//   spin_gram: G[p][t][s1][s2] = sum_{m,c} conj(A_p(t,m,s1,c)) B_p(t,m,s2,c)
//              (spin-resolved timeslice inner products of solution pairs)
// Spinor fields are canonical complex128 [T][Z][Y][X][4][3]; V is [T][nev][L^3][3].
#include "laplace.h"

namespace dlma {

__device__ __forceinline__ double2 cjm(double2 a, double2 b) { return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }

// one block per (k-group of 4, t, f)
__global__ void __launch_bounds__(256) k_tproj(const double2* __restrict__ Vall, const double2* const* __restrict__ fields,
                                               long L3, int nev, int T, double2* __restrict__ P) {
    __shared__ double lds[4];
    int k0 = blockIdx.x * 4, t = blockIdx.y, f = blockIdx.z;
    const double2* phi = fields[f] + (long)t * L3 * 12;
    const double2* Vt = Vall + (long)t * nev * L3 * 3;
    double2 acc[4][4];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0, 0);
    for (long m = threadIdx.x; m < L3; m += 256) {
        double2 ps[12];
        for (int i = 0; i < 12; ++i) ps[i] = phi[m * 12 + i];
        for (int kk = 0; kk < 4; ++kk) {
            if (k0 + kk >= nev) break;
            const double2* v = Vt + ((long)(k0 + kk) * L3 + m) * 3;
            double2 v0 = v[0], v1 = v[1], v2 = v[2];
            for (int sp = 0; sp < 4; ++sp) {
                double2 a = cjm(v0, ps[sp * 3]), b = cjm(v1, ps[sp * 3 + 1]), c = cjm(v2, ps[sp * 3 + 2]);
                acc[kk][sp].x += a.x + b.x + c.x;
                acc[kk][sp].y += a.y + b.y + c.y;
            }
        }
    }
    for (int kk = 0; kk < 4; ++kk) {
        if (k0 + kk >= nev) break;  // uniform
        for (int sp = 0; sp < 4; ++sp) {
            double re = block_sum<256>(acc[kk][sp].x, lds);
            double im = block_sum<256>(acc[kk][sp].y, lds);
            if (threadIdx.x == 0) P[(((long)f * T + t) * nev + k0 + kk) * 4 + sp] = make_double2(re, im);
        }
    }
}

hipError_t launch_tproj(const double2* Vall, const double2* const* fields, int nf, const Geo& g, int nev, double2* P,
                        hipStream_t s) {
    long L3 = (long)g.Z * g.Y * g.X;
    if (nf <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tproj, dim3((nev + 3) / 4, g.T, nf), dim3(256), 0, s, Vall, fields, L3, nev, g.T, P);
    return hipGetLastError();
}

// one block per (t, pair)
__global__ void __launch_bounds__(256) k_spin_gram(const double2* const* __restrict__ A, const double2* const* __restrict__ B,
                                                   long L3, int T, double2* __restrict__ G) {
    __shared__ double lds[4];
    int t = blockIdx.x, p = blockIdx.y;
    const double2* a = A[p] + (long)t * L3 * 12;
    const double2* b = B[p] + (long)t * L3 * 12;
    double2 acc[16];
    for (int i = 0; i < 16; ++i) acc[i] = make_double2(0, 0);
    for (long m = threadIdx.x; m < L3; m += 256) {
        double2 av[12], bv[12];
        for (int i = 0; i < 12; ++i) { av[i] = a[m * 12 + i]; bv[i] = b[m * 12 + i]; }
        for (int s1 = 0; s1 < 4; ++s1)
            for (int s2 = 0; s2 < 4; ++s2)
                for (int c = 0; c < 3; ++c) {
                    double2 q = cjm(av[s1 * 3 + c], bv[s2 * 3 + c]);
                    acc[s1 * 4 + s2].x += q.x;
                    acc[s1 * 4 + s2].y += q.y;
                }
    }
    for (int i = 0; i < 16; ++i) {
        double re = block_sum<256>(acc[i].x, lds);
        double im = block_sum<256>(acc[i].y, lds);
        if (threadIdx.x == 0) G[((long)p * T + t) * 16 + i] = make_double2(re, im);
    }
}

hipError_t launch_spin_gram(const double2* const* A, const double2* const* B, int npair, const Geo& g, double2* G,
                            hipStream_t s) {
    long L3 = (long)g.Z * g.Y * g.X;
    if (npair <= 0) return hipSuccess;
    for (int p0 = 0; p0 < npair; p0 += 65535) {
        int np = npair - p0 < 65535 ? npair - p0 : 65535;
        hipLaunchKernelGGL(k_spin_gram, dim3(g.T, np), dim3(256), 0, s, A + p0, B + p0, L3, g.T, G + (long)p0 * g.T * 16);
    }
    return hipGetLastError();
}

}  // namespace dlma
