// Shared device/host definitions of the dlma library: precision traits, the
// even-odd site geometry, pair storage (one complex number per element),
// spinor-field views and the per-job launch descriptors.
//
// Internal layouts (structure of arrays, site index fastest, one launch
// touches consecutive sites with consecutive lanes):
//   links       [parity][mu][9 = a*3+b][Vh]         pairs
//   clover      [block 0/1][18][Vh] per parity       pairs: 3 pairs of diagonal
//               reals (d0,d1),(d2,d3),(d4,d5) then the 15 lower entries l_ij,
//               i > j, ordered (1,0),(2,0),(2,1),(3,0),...,(5,4)
//   half field  [rhs][12 = spin*3+colour][Vh]        pairs; FP16 fields instead
//               [rhs][3][Vh][4]: components 4g .. 4g+3 of a site in one 16-byte
//               group g (one 128-bit load), plus [rhs][Vh] FP32 scales
//   FP16 links  [parity][mu][row a][Vh][3]           words (one 96-bit load per row)
//   FP16 clover [block][5][Vh][4]                    words: the 18 of a block in
//               groups of 4 (the last group padded with 2 zero words)
//   full field  [rhs][parity][12][Vh]                FP64 pairs
// Even-odd index of site (t,z,y,x): parity = (t+z+y+x) & 1,
//   cb = ((t*Z + z)*Y + y)*(X/2) + x/2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define HD __host__ __device__ __forceinline__

namespace dlma {

enum Prec { P64 = 0, P32 = 1, P16 = 2, PB16 = 3 };

template <int P> struct PT;
template <> struct PT<P64> { using S = double2; using R = double; };
template <> struct PT<P32> { using S = float2; using R = float; };
template <> struct PT<P16> { using S = uint32_t; using R = float; };   // 2 x binary16, re low
template <> struct PT<PB16> { using S = uint32_t; using R = float; };  // 2 x bfloat16, re low

inline size_t pair_bytes(int p) { return p == P64 ? 16 : (p == P32 ? 8 : 4); }

// ---------------------------------------------------------------- scalar conversions

HD float bf16_to_f(uint32_t bits16) { return __builtin_bit_cast(float, bits16 << 16); }
HD uint32_t f_to_bf16(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return u >> 16;
}
HD float h_to_f(uint32_t bits16) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)bits16);
}
HD uint32_t f_to_h(float f) { return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)f); }

// Scheduling fences around a group of vector-memory stores with more than 64 bits of
// data each, closed by two wait states.  Such a store reads its data registers after
// it issues; a vector ALU instruction that overwrites them in the next cycle corrupts
// the stored value, and the compiler in use emits that sequence without the wait
// state (seen as stored values that changed from run to run).  The build checks the
// machine code of every kernel for the pattern.
HD void wide_store_begin() {
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_sched_barrier(0);
#endif
}
HD void wide_store_end() {
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_sched_barrier(0);
    __asm__ volatile("s_nop 1");
    __builtin_amdgcn_sched_barrier(0);
#endif
}

// load / store one complex element
template <int P> HD void ldp(const typename PT<P>::S* a, size_t i, typename PT<P>::R& re, typename PT<P>::R& im);
// FP64 fields are global memory: addressed as such, the loads and stores are
// global_* instructions, which count against the vector-memory counter only (a flat
// access also counts against the LDS/scalar counter that the scalar loads wait on).
#if defined(__HIP_DEVICE_COMPILE__)
typedef const __attribute__((address_space(1))) double2* GlobalD2;
typedef __attribute__((address_space(1))) double2* GlobalD2w;
#endif
template <> HD void ldp<P64>(const double2* a, size_t i, double& re, double& im) {
#if defined(__HIP_DEVICE_COMPILE__)
    const double2 v = ((GlobalD2)a)[i];
#else
    const double2 v = a[i];
#endif
    re = v.x;
    im = v.y;
}
template <> HD void ldp<P32>(const float2* a, size_t i, float& re, float& im) { float2 v = a[i]; re = v.x; im = v.y; }
template <> HD void ldp<P16>(const uint32_t* a, size_t i, float& re, float& im) { uint32_t v = a[i]; re = h_to_f(v & 0xffffu); im = h_to_f(v >> 16); }
template <> HD void ldp<PB16>(const uint32_t* a, size_t i, float& re, float& im) { uint32_t v = a[i]; re = bf16_to_f(v & 0xffffu); im = bf16_to_f(v >> 16); }

template <int P> HD void stp(typename PT<P>::S* a, size_t i, typename PT<P>::R re, typename PT<P>::R im);
template <> HD void stp<P64>(double2* a, size_t i, double re, double im) {
#if defined(__HIP_DEVICE_COMPILE__)
    ((GlobalD2w)a)[i] = make_double2(re, im);
#else
    a[i] = make_double2(re, im);
#endif
}
template <> HD void stp<P32>(float2* a, size_t i, float re, float im) { a[i] = make_float2(re, im); }
template <> HD void stp<P16>(uint32_t* a, size_t i, float re, float im) { a[i] = f_to_h(re) | (f_to_h(im) << 16); }
template <> HD void stp<PB16>(uint32_t* a, size_t i, float re, float im) { a[i] = f_to_bf16(re) | (f_to_bf16(im) << 16); }

// ---------------------------------------------------------------- geometry

struct Geo {
    int T, Z, Y, X, Xh, Vh;
    uint64_t mXh, mY, mZ;  // magic multipliers: n / d == (n * m) >> 36 for n < 2^24, d <= 4096
};

// Division by a lattice extent via a precomputed multiplier m = floor(2^36/d) + 1:
// (n m) >> 36 = n/d + n e/(d 2^36) with 0 < e <= d, exact while n d < 2^36.
HD uint32_t mdiv(uint32_t n, uint64_t m) { return (uint32_t)(((uint64_t)n * m) >> 36); }
inline uint64_t magic36(uint32_t d) { return ((((uint64_t)1) << 36) / d) + 1; }

inline Geo make_geo(const int dims[4]) {
    Geo g;
    g.T = dims[0]; g.Z = dims[1]; g.Y = dims[2]; g.X = dims[3];
    g.Xh = g.X / 2;
    g.Vh = g.T * g.Z * g.Y * g.Xh;
    g.mXh = magic36(g.Xh); g.mY = magic36(g.Y); g.mZ = magic36(g.Z);
    return g;
}

// Neighbour table of one site: index 2*mu + 0 = forward, 2*mu + 1 = backward
// (opposite parity), mu = 0:t 1:x 2:y 3:z.
struct Nbr { int n[8]; };

HD Nbr neighbours(const Geo& g, int par, int cb) {
    uint32_t xh = cb - g.Xh * mdiv(cb, g.mXh);
    uint32_t r1 = mdiv(cb, g.mXh);
    uint32_t y = r1 - g.Y * mdiv(r1, g.mY);
    uint32_t r2 = mdiv(r1, g.mY);
    uint32_t z = r2 - g.Z * mdiv(r2, g.mZ);
    uint32_t t = mdiv(r2, g.mZ);
    int x = 2 * (int)xh + (int)((t + z + y + par) & 1u);
    int base = cb - (int)xh;
    Nbr o;
    int sY = g.Xh, sZ = g.Y * g.Xh, sT = g.Z * g.Y * g.Xh;
    int tp = (int)t + 1 == g.T ? 0 : (int)t + 1, tm = t == 0 ? g.T - 1 : (int)t - 1;
    int zp = (int)z + 1 == g.Z ? 0 : (int)z + 1, zm = z == 0 ? g.Z - 1 : (int)z - 1;
    int yp = (int)y + 1 == g.Y ? 0 : (int)y + 1, ym = y == 0 ? g.Y - 1 : (int)y - 1;
    int xp = x + 1 == g.X ? 0 : x + 1, xm = x == 0 ? g.X - 1 : x - 1;
    o.n[0] = cb + (tp - (int)t) * sT;
    o.n[1] = cb + (tm - (int)t) * sT;
    o.n[2] = base + (xp >> 1);
    o.n[3] = base + (xm >> 1);
    o.n[4] = cb + (yp - (int)y) * sY;
    o.n[5] = cb + (ym - (int)y) * sY;
    o.n[6] = cb + (zp - (int)z) * sZ;
    o.n[7] = cb + (zm - (int)z) * sZ;
    return o;
}

// Whether source r may be nonzero at timeslice t, dilated by tdil timeslices either
// way (periodic); true without support flags.
HD bool tsup_any(const int* tsup, int T, int r, int t, int tdil) {
    if (!tsup) return true;
    const int* f = tsup + (size_t)r * T;
    int any = f[t];
    for (int d = 1; d <= tdil; ++d) any |= f[t + d < T ? t + d : t + d - T] | f[t - d >= 0 ? t - d : t - d + T];
    return any != 0;
}

// Reach of the first pass's Krylov vectors.  From x = 0 the first inner solve starts
// on the Schur source, which is nonzero only within 1 timeslice of the source's
// support, and each application of the Schur operator (two hops) widens that by 2:
// after k iterations the s of BiCGStab is nonzero only within 3 + 4k timeslices and
// the updated x, r, p within 5 + 4k.  tdist[r][t] is the distance (periodic) from t
// to the nearest timeslice where source r is nonzero, or 0 everywhere once the
// vectors are dense (later passes); the FP16 vector steps skip the sites beyond the
// reach, whose values are exact zeros.  (The stencils do not: a block that exits
// early still costs its dispatch and the loads of its decision, about what the
// skipped work saves.)
HD bool in_reach(const int* tdist, const int* titer, int T, int r, int t, int c) {
    if (!tdist) return true;
    return tdist[(size_t)r * T + t] <= c + 4 * titer[r];
}

// ---------------------------------------------------------------- field views

// A set of nrhs half-lattice spinor fields: element (r, comp, site) at
// v[r*rs + comp*Vh + site]; FP16 fields carry a per-(r, site) scale at nrm[r*ns + site].
template <int P> struct SF {
    typename PT<P>::S* v;
    float* nrm;
    long rs;
    long ns;
};

// word w (0..11, = component) of site cb in an FP16 field's row r: group w/4, slot w%4
HD size_t f16_word(const SF<P16>& f, int Vh, int r, int cb, int w) {
    return (size_t)r * f.rs + ((size_t)(w >> 2) * Vh + cb) * 4 + (w & 3);
}

template <int P, class R> HD void load_spinor(const SF<P>& f, int Vh, int r, int cb, R s[24]) {
    if constexpr (P == P16) {
        const R n = (R)f.nrm[(size_t)r * f.ns + cb];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const uint32_t w = f.v[f16_word(f, Vh, r, cb, c)];
            s[2 * c] = (R)h_to_f(w & 0xffffu) * n;
            s[2 * c + 1] = (R)h_to_f(w >> 16) * n;
        }
    } else {
        const typename PT<P>::S* b = f.v + (size_t)r * f.rs + cb;
#pragma unroll
        for (int c = 0; c < 12; ++c) ldp<P>(b, (size_t)c * Vh, s[2 * c], s[2 * c + 1]);
    }
}

// An FP16-stored site widened to FP64 and multiplied by fac: component = binary16
// value * (scale * fac), where the binary16 value times the FP32 scale is exact in
// FP64 and (scale * fac) is rounded once.  Every FP64 consumer of the same stored
// field (the accumulation into x, whether its own kernel or fused into the next
// residual, and the odd-site reconstruction) goes through f16_factor and f16_widen,
// so all of them see bit-identical values.  The 16-byte word groups load as one
// 128-bit access each.
HD double f16_factor(const SF<P16>& f, int r, int cb, double fac) { return (double)f.nrm[(size_t)r * f.ns + cb] * fac; }
HD double f16_widen(uint32_t bits16, double n) { return (double)h_to_f(bits16) * n; }
#if defined(__HIP_DEVICE_COMPILE__)
typedef const __attribute__((address_space(1))) uint4* GlobalU4;
#else
typedef const uint4* GlobalU4;
#endif

HD void load_spinor16_f64(const SF<P16>& f, int Vh, int r, int cb, double fac, double s[24]) {
    const double n = f16_factor(f, r, cb, fac);
    const GlobalU4 q = (GlobalU4)(f.v + (size_t)r * f.rs);
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        const uint4 v = q[(size_t)g * Vh + cb];
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            s[8 * g + 2 * k] = f16_widen(w[k] & 0xffffu, n);
            s[8 * g + 2 * k + 1] = f16_widen(w[k] >> 16, n);
        }
    }
}

// The same for the six components of half blk (spins 2 blk, 2 blk + 1), added to s.
HD void add_half16_f64(const SF<P16>& f, int Vh, int r, int cb, int blk, double fac, double s[12]) {
    const double n = f16_factor(f, r, cb, fac);
    const GlobalU4 q = (GlobalU4)(f.v + (size_t)r * f.rs);
    // components 6 blk .. 6 blk + 5 lie in word groups blk and blk + 1
    const uint4 v0 = q[(size_t)blk * Vh + cb], v1 = q[(size_t)(blk + 1) * Vh + cb];
    const uint32_t w[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
    const int o = blk == 0 ? 0 : 2;  // first component of the half within the two groups
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        s[2 * k] += f16_widen(w[o + k] & 0xffffu, n);
        s[2 * k + 1] += f16_widen(w[o + k] >> 16, n);
    }
}

template <int P, class R> HD void store_spinor(const SF<P>& f, int Vh, int r, int cb, const R s[24]) {
    if constexpr (P == P16) {
        float m = 0.f;
#pragma unroll
        for (int i = 0; i < 24; ++i) m = fmaxf(m, fabsf((float)s[i]));
        // Sites whose largest component is below 1e-30 are stored as zero: the inner
        // solver works on unit-norm vectors, so such sites are rounding residue at the
        // edge of a propagating support, and 1/m would overflow near FP32's denormal range.
        if (!(m >= 1e-30f)) m = 0.f;
        float inv = m > 0.f ? 1.0f / m : 0.f;
        f.nrm[(size_t)r * f.ns + cb] = m;
        uint32_t w[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) w[c] = f_to_h((float)s[2 * c] * inv) | (f_to_h((float)s[2 * c + 1] * inv) << 16);
        // the three groups of four words compile to 128-bit stores
        wide_store_begin();
#pragma unroll
        for (int c = 0; c < 12; ++c) f.v[f16_word(f, Vh, r, cb, c)] = w[c];
        wide_store_end();
    } else {
        typename PT<P>::S* b = f.v + (size_t)r * f.rs + cb;
#pragma unroll
        for (int c = 0; c < 12; ++c) stp<P>(b, (size_t)c * Vh, (typename PT<P>::R)s[2 * c], (typename PT<P>::R)s[2 * c + 1]);
    }
}

// ---------------------------------------------------------------- stencil pieces

// 3x3 link, row-major complex: u[2*(a*3+b)], u[2*(a*3+b)+1]
template <int P, class R> HD void load_link(const typename PT<P>::S* U, int Vh, int par, int mu, int cb, R u[18]) {
    const typename PT<P>::S* b = U + ((size_t)(par * 4 + mu) * 9) * Vh + cb;
#pragma unroll
    for (int k = 0; k < 9; ++k) ldp<P>(b, (size_t)k * Vh, u[2 * k], u[2 * k + 1]);
}

// g = U h (DAG = false) or U^dag h (DAG = true) for two half-spin components h[2][3]
template <bool DAG, class R> HD void su3_mul2(const R u[18], const R h[12], R gout[12]) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            R re = 0, im = 0;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                R ur, ui;
                if (!DAG) { ur = u[2 * (a * 3 + b)]; ui = u[2 * (a * 3 + b) + 1]; }
                else { ur = u[2 * (b * 3 + a)]; ui = -u[2 * (b * 3 + a) + 1]; }
                R hr = h[2 * (s * 3 + b)], hi = h[2 * (s * 3 + b) + 1];
                re += ur * hr - ui * hi;
                im += ur * hi + ui * hr;
            }
            gout[2 * (s * 3 + a)] = re;
            gout[2 * (s * 3 + a) + 1] = im;
        }
}

// One hopping term: acc += (1 -/+ g_mu) U psi(neighbour), with the spin
// projection written out for the chiral basis.  FWD: (1 - g_mu) U_mu(x) psi(x+mu);
// backward: (1 + g_mu) U_mu(x-mu)^dag psi(x-mu).  G5IN multiplies psi by g5 first.
template <int MU, bool FWD, bool G5IN, class R> HD void hop_term(const R u[18], const R psi[24], R acc[24]) {
    const R s5 = G5IN ? (R)-1 : (R)1;
    R h[12];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R p0r = psi[2 * (0 * 3 + a)], p0i = psi[2 * (0 * 3 + a) + 1];
        R p1r = psi[2 * (1 * 3 + a)], p1i = psi[2 * (1 * 3 + a) + 1];
        R p2r = s5 * psi[2 * (2 * 3 + a)], p2i = s5 * psi[2 * (2 * 3 + a) + 1];
        R p3r = s5 * psi[2 * (3 * 3 + a)], p3i = s5 * psi[2 * (3 * 3 + a) + 1];
        R h0r, h0i, h1r, h1i;
        if (MU == 0) {
            if (FWD) { h0r = p0r + p2r; h0i = p0i + p2i; h1r = p1r + p3r; h1i = p1i + p3i; }
            else { h0r = p0r - p2r; h0i = p0i - p2i; h1r = p1r - p3r; h1i = p1i - p3i; }
        } else if (MU == 1) {  // i*psi = (-im, re)
            if (FWD) { h0r = p0r - p3i; h0i = p0i + p3r; h1r = p1r - p2i; h1i = p1i + p2r; }
            else { h0r = p0r + p3i; h0i = p0i - p3r; h1r = p1r + p2i; h1i = p1i - p2r; }
        } else if (MU == 2) {
            if (FWD) { h0r = p0r + p3r; h0i = p0i + p3i; h1r = p1r - p2r; h1i = p1i - p2i; }
            else { h0r = p0r - p3r; h0i = p0i - p3i; h1r = p1r + p2r; h1i = p1i + p2i; }
        } else {
            if (FWD) { h0r = p0r - p2i; h0i = p0i + p2r; h1r = p1r + p3i; h1i = p1i - p3r; }
            else { h0r = p0r + p2i; h0i = p0i - p2r; h1r = p1r - p3i; h1i = p1i + p3r; }
        }
        h[2 * a] = h0r; h[2 * a + 1] = h0i;
        h[2 * (3 + a)] = h1r; h[2 * (3 + a) + 1] = h1i;
    }
    R g[12];
    su3_mul2<!FWD>(u, h, g);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R g0r = g[2 * a], g0i = g[2 * a + 1], g1r = g[2 * (3 + a)], g1i = g[2 * (3 + a) + 1];
        acc[2 * (0 * 3 + a)] += g0r; acc[2 * (0 * 3 + a) + 1] += g0i;
        acc[2 * (1 * 3 + a)] += g1r; acc[2 * (1 * 3 + a) + 1] += g1i;
        R d2r, d2i, d3r, d3i;
        if (MU == 0) {
            if (FWD) { d2r = g0r; d2i = g0i; d3r = g1r; d3i = g1i; }
            else { d2r = -g0r; d2i = -g0i; d3r = -g1r; d3i = -g1i; }
        } else if (MU == 1) {  // fwd: (-i g1, -i g0); bwd: (i g1, i g0);  -i z = (im, -re)
            if (FWD) { d2r = g1i; d2i = -g1r; d3r = g0i; d3i = -g0r; }
            else { d2r = -g1i; d2i = g1r; d3r = -g0i; d3i = g0r; }
        } else if (MU == 2) {  // fwd: (-g1, g0); bwd: (g1, -g0)
            if (FWD) { d2r = -g1r; d2i = -g1i; d3r = g0r; d3i = g0i; }
            else { d2r = g1r; d2i = g1i; d3r = -g0r; d3i = -g0i; }
        } else {  // fwd: (-i g0, i g1); bwd: (i g0, -i g1)
            if (FWD) { d2r = g0i; d2i = -g0r; d3r = -g1i; d3i = g1r; }
            else { d2r = -g0i; d2i = g0r; d3r = g1i; d3i = -g1r; }
        }
        acc[2 * (2 * 3 + a)] += d2r; acc[2 * (2 * 3 + a) + 1] += d2i;
        acc[2 * (3 * 3 + a)] += d3r; acc[2 * (3 * 3 + a) + 1] += d3i;
    }
}

// y = H x for one packed Hermitian 6x6 block (36 reals) and a 6-vector
template <class R> HD void herm6(const R c[36], const R* x, R* y) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        y[2 * i] = c[i] * x[2 * i];
        y[2 * i + 1] = c[i] * x[2 * i + 1];
    }
    int k = 0;
#pragma unroll
    for (int i = 1; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < i; ++j, ++k) {
            R lr = c[6 + 2 * k], li = c[6 + 2 * k + 1];
            R xjr = x[2 * j], xji = x[2 * j + 1], xir = x[2 * i], xii = x[2 * i + 1];
            y[2 * i] += lr * xjr - li * xji;
            y[2 * i + 1] += lr * xji + li * xjr;
            y[2 * j] += lr * xir + li * xii;
            y[2 * j + 1] += lr * xii - li * xir;
        }
}

template <int P, class R> HD void load_clover_block(const typename PT<P>::S* C, int Vh, int blk, int cb, R c[36]) {
    const typename PT<P>::S* b = C + (size_t)blk * 18 * Vh + cb;
#pragma unroll
    for (int q = 0; q < 18; ++q) ldp<P>(b, (size_t)q * Vh, c[2 * q], c[2 * q + 1]);
}

}  // namespace dlma
