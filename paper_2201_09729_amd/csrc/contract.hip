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


// ---------------------------------------------------------------- backward of the contractions
//
// Every correlator piece is a sesquilinear form sum <A, M X_t B>_t in the solution
// fields of one source group (four spin-diluted solutions, plus their (1 - box)
// partners for noise).  Its gradient field on timeslice t is therefore
//   grad(t, x) = W1(t) F(t, x) + WP(t) (box(t) F)(t, x),
// with F the group's input fields stacked with their spin components, W1 and WP spin
// matrices that combine the loss weights, Gamma, g5 and the normalisations (the same
// for every group), and box(t) F = sum_k v_k(t) tau_k, tau = V(t)^dag F.  The host
// folds WP into tau' = WP tau; this kernel forms W1 F + sum_k v_k tau'_k for one
// output chunk (four output fields of one group) at 256 rows (site, colour) of one
// timeslice per block.  W1 rows and tau' of the chunk are staged in LDS.
__global__ void __launch_bounds__(256) k_corr_grad(CorrGradArgs a) {
    __shared__ double2 w1s[16 * 32];  // W1 rows of the chunk's 16 outputs, over <= 32 inputs
    __shared__ double2 tps[64 * 16];  // tau'[k][16 outputs] for 64 modes at a time
    const int t = blockIdx.y, z = blockIdx.z;
    const bool noise = z < 2 * a.nnoise;
    const int grp = noise ? z >> 1 : z - 2 * a.nnoise;
    const int half = noise ? (z & 1) : 0;
    const int nin = noise ? 32 : 16;  // input (field, spin) columns of a group
    const int ta = a.tact[t];         // uniform: the block's timeslice carries weights or not
    const long L3 = a.L3;
    const long row = (long)blockIdx.x * 256 + threadIdx.x;
    const bool valid = row < L3 * 3;
    const long x = valid ? row / 3 : 0;
    const int c = (int)(valid ? row - x * 3 : 0);
    const long site = ((long)t * L3 + x) * 12 + c;  // offset of (spin 0, colour c) in a field
    double2 acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = make_double2(0.0, 0.0);
    if (ta >= 0) {
        const double2* W1 = noise ? a.W1n + ((long)t * 32 + half * 16) * 32 : a.W1d + (long)t * 16 * 16;
        for (int i = threadIdx.x; i < 16 * nin; i += 256) w1s[i] = W1[i];
        __syncthreads();
        if (valid) {
            for (int j = 0; j < nin / 4; ++j) {
                const double2* f = noise ? (j < 4 ? a.phi + ((long)grp * 4 + j) * a.fs : a.phibar + ((long)grp * 4 + j - 4) * a.fs)
                                         : a.dist + ((long)grp * 4 + j) * a.fs;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const double2 v = f[site + b * 3];
                    const int col = j * 4 + b;
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const double2 w = w1s[q * nin + col];
                        acc[q].x += w.x * v.x - w.y * v.y;
                        acc[q].y += w.x * v.y + w.y * v.x;
                    }
                }
            }
        }
        const double2* tp = noise ? a.taun + (((long)grp * a.nact + ta) * a.nev) * 32 + half * 16
                                  : a.taud + (((long)grp * a.nact + ta) * a.nev) * 16;
        const int tstride = noise ? 32 : 16;
        const double2* vk = a.Vall + (long)t * a.nev * L3 * 3 + (valid ? row : 0);
        for (int k0 = 0; k0 < a.nev; k0 += 64) {
            const int nk = a.nev - k0 < 64 ? a.nev - k0 : 64;
            __syncthreads();  // the previous chunk (or W1) has been read by every thread
            for (int i = threadIdx.x; i < nk * 16; i += 256) tps[i] = tp[(long)(k0 + (i >> 4)) * tstride + (i & 15)];
            __syncthreads();
            if (valid) {
                for (int k = 0; k < nk; ++k) {
                    const double2 v = vk[(long)(k0 + k) * L3 * 3];
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const double2 w = tps[k * 16 + q];
                        acc[q].x += w.x * v.x - w.y * v.y;
                        acc[q].y += w.x * v.y + w.y * v.x;
                    }
                }
            }
        }
    }
    if (!valid) return;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double2* o = noise ? (half == 0 ? a.gphi : a.gphibar) + ((long)grp * 4 + i) * a.fs : a.gdist + ((long)grp * 4 + i) * a.fs;
#pragma unroll
        for (int s = 0; s < 4; ++s) o[site + s * 3] = acc[i * 4 + s];
    }
}

hipError_t launch_corr_grad(const CorrGradArgs& a, int T, hipStream_t s) {
    const int nchunk = 2 * a.nnoise + a.ndist;  // grid z: the callers keep it below 65536
    if (nchunk <= 0) return hipSuccess;
    if (nchunk > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_corr_grad, dim3((unsigned)((a.L3 * 3 + 255) / 256), T, nchunk), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace dlma
