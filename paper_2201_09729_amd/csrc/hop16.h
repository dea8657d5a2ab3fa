// Per-site body of the stencil kernels for FP16-stored fields.
//
// Same operator and flags as the generic body in hop.h; what differs is how the
// binary16 data reaches the FP32 arithmetic, which decides the speed once many
// right-hand sides share each link (the multi-RHS stencil is bound by vector
// instruction issue, not by HBM):
//   * every field is read through buffer loads whose per-lane operand is just the
//     site's byte offset (component and right-hand-side offsets travel in scalar
//     registers), 128 or 96 bits per load: the FP16 layouts keep four components
//     of a site (spinors, clover) or one link row together, because the memory
//     pipeline's cost is per load instruction, not per byte;
//   * the SU(3) products run on packed binary16 pairs: the spin projection
//     h = a +- b (or a +- i b) is formed in binary16 (one rounding, at storage
//     precision) and each complex product is two v_dot2 instructions (exact
//     binary16 products, FP32 accumulation), half the instructions of FP32 FMAs;
//   * clover entries and own-site spinors enter mixed-precision FMAs directly
//     (gfx950 reads an f16 operand, low or high half, inside an FP32 FMA), so
//     nothing is converted one value at a time;
//   * the per-(site, RHS) scale of an FP16 spinor and the kernel's coefficients
//     (ch, ca, -alpha) are folded into the FMAs that accumulate the result
//     instead of being multiplied into every component.
// Accumulation is FP32 throughout.
#pragma once
#include "common.h"

namespace dlma {

// ---------------------------------------------------------------- word access

// A read-only or writable region of 32-bit words.  On the device it is a buffer
// resource; word (lane byte offset v, uniform byte offset s) sits at base + v + s.
struct WSrc {
#if defined(__HIP_DEVICE_COMPILE__)
    __amdgpu_buffer_rsrc_t r;
#else
    char* p;
#endif
};

HD WSrc wsrc(const void* base, uint32_t bytes) {
    WSrc s;
#if defined(__HIP_DEVICE_COMPILE__)
    // third descriptor word of a raw (unswizzled, stride 0) 32-bit buffer on gfx9-class parts
    s.r = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
#else
    (void)bytes;
    s.p = (char*)const_cast<void*>(base);
#endif
    return s;
}

// Cache policy of a buffer access: 0 = default, NT = non-temporal (streamed, not
// kept in L2).  Stores and single-use loads of the own site stream, so the L2
// keeps the data that is reused: links, clover and the neighbour spinors.
enum { CP_DEFAULT = 0, CP_NT = 2 };

template <int CP = CP_DEFAULT> HD uint32_t wld(const WSrc& s, uint32_t v, uint32_t u) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_raw_buffer_load_b32(s.r, (int)v, (int)u, CP);
#else
    return *(const uint32_t*)(s.p + (size_t)v + u);
#endif
}

HD void wst(const WSrc& s, uint32_t v, uint32_t u, uint32_t w) {
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_raw_buffer_store_b32(w, s.r, (int)v, (int)u, CP_NT);
#else
    *(uint32_t*)(s.p + (size_t)v + u) = w;
#endif
}

template <int CP = CP_DEFAULT> HD float wldf(const WSrc& s, uint32_t v, uint32_t u) {
    return __builtin_bit_cast(float, wld<CP>(s, v, u));
}

// 128- and 96-bit accesses (one instruction each): the memory pipeline's cost per
// instruction, not per byte, bounds the multi-RHS stencil, so every field is laid
// out for the widest load that fits it.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));

template <int CP = CP_DEFAULT> HD u32x4 wld4(const WSrc& s, uint32_t v, uint32_t u) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_raw_buffer_load_b128(s.r, (int)v, (int)u, CP);
#else
    return *(const u32x4*)(s.p + (size_t)v + u);
#endif
}

HD u32x3 wld3(const WSrc& s, uint32_t v, uint32_t u) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_raw_buffer_load_b96(s.r, (int)v, (int)u, 0);
#else
    const uint32_t* q = (const uint32_t*)(s.p + (size_t)v + u);
    return (u32x3){q[0], q[1], q[2]};
#endif
}

HD void wst4(const WSrc& s, uint32_t v, uint32_t u, u32x4 w) {
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_raw_buffer_store_b128(w, s.r, (int)v, (int)u, CP_NT);
#else
    *(u32x4*)(s.p + (size_t)v + u) = w;
#endif
}

// binary16 halves of a word, widened where they are consumed
HD float lo16(uint32_t w) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu)); }
HD float hi16(uint32_t w) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16)); }

// One FP16 spinor field of the job for right-hand side r: components and the scale.
struct F16Field {
    WSrc v, n;
};
HD F16Field f16_field(const SF<P16>& f, int Vh, int r) {
    F16Field o;
    o.v = wsrc(f.v + (size_t)r * f.rs, 12u * 4u * (uint32_t)Vh);
    o.n = wsrc(f.nrm + (size_t)r * f.ns, 4u * (uint32_t)Vh);
    return o;
}

// The 12 words of one site: three 16-byte groups (layout [3][Vh][4]); site16 = 16 site,
// G16 = 16 Vh bytes per group plane.
template <int CP = CP_DEFAULT> HD void load_words(const F16Field& f, uint32_t site16, uint32_t G16, uint32_t w[12]) {
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        const u32x4 v = wld4<CP>(f.v, site16, (uint32_t)g * G16);
        w[4 * g] = v.x; w[4 * g + 1] = v.y; w[4 * g + 2] = v.z; w[4 * g + 3] = v.w;
    }
}

// Link U_mu at parity par, site offset site12 = 12 site: rows a = 0..2 of three words
// each (layout [par][mu][3][Vh][3]); R12 = 12 Vh bytes per row plane.
HD void load_link16(const WSrc& U, uint32_t site12, uint32_t R12, int par, int mu, uint32_t u[9]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const u32x3 v = wld3(U, site12, (uint32_t)((par * 4 + mu) * 3 + a) * R12);
        u[3 * a] = v.x; u[3 * a + 1] = v.y; u[3 * a + 2] = v.z;
    }
}

// ---------------------------------------------------------------- spin structure

// Chiral-basis spin projection of the hop in direction MU (see hop_term in
// common.h, which this restates in table form):
//   h_s = p_s + c_s p_{Q_s}       (s = 0, 1)
//   lower spins: d_2 = e_2 g_{R_2}, d_3 = e_3 g_{R_3},  g = U' h
// with coefficient codes 0: +1, 1: -1, 2: +i, 3: -i.  The backward hop negates
// every c and e; g5 on the input negates c, g5 on the output negates e.
template <int MU> struct Spin {
    static constexpr int Q0 = (MU == 0 || MU == 3) ? 2 : 3;
    static constexpr int Q1 = 5 - Q0;
    static constexpr int C0 = MU == 0 ? 0 : (MU == 1 ? 2 : (MU == 2 ? 0 : 2));
    static constexpr int C1 = MU == 0 ? 0 : (MU == 1 ? 2 : (MU == 2 ? 1 : 3));
    static constexpr int R2 = (MU == 0 || MU == 3) ? 0 : 1;
    static constexpr int R3 = 1 - R2;
    static constexpr int E2 = MU == 0 ? 0 : (MU == 1 ? 3 : (MU == 2 ? 1 : 3));
    static constexpr int E3 = MU == 0 ? 0 : (MU == 1 ? 3 : (MU == 2 ? 0 : 2));
};

// Packed binary16 pairs and the spin projection in the two forms the dot products
// of the SU(3) multiplication need.  For h = p + c q (complex, formed in binary16
// with one rounding, |h| <= 2 since stored spinors are scaled to magnitude <= 1):
//   forward hop  (U h):     w1 = (hr, -hi), w2 = (hi, hr)
//   backward hop (U^dag h): w1 = (hr,  hi), w2 = (hi, -hr)
// so that with u = (ur, ui) of one link entry, dot(u, w1) and dot(u, w2) are the
// real and imaginary parts of u h (forward) or conj(u) h (backward).  Each dot
// product is one v_dot2 instruction: two exact binary16 products summed in FP32.
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
HD half2_t as_h2(uint32_t w) { return __builtin_bit_cast(half2_t, w); }

template <int C, bool FWD> HD void proj_h2(uint32_t pw, uint32_t qw, half2_t& w1, half2_t& w2) {
    const half2_t p = as_h2(pw), q = as_h2(qw);
    if (FWD) {
        const half2_t pa = (half2_t){p.x, -p.y}, pb = (half2_t){p.y, p.x};
        if (C == 0) { w1 = pa + (half2_t){q.x, -q.y}; w2 = pb + (half2_t){q.y, q.x}; }
        if (C == 1) { w1 = pa - (half2_t){q.x, -q.y}; w2 = pb - (half2_t){q.y, q.x}; }
        if (C == 2) { w1 = pa + (half2_t){-q.y, -q.x}; w2 = pb + (half2_t){q.x, -q.y}; }
        if (C == 3) { w1 = pa + (half2_t){q.y, q.x}; w2 = pb + (half2_t){-q.x, q.y}; }
    } else {
        const half2_t pb = (half2_t){p.y, -p.x};
        if (C == 0) { w1 = p + q; w2 = pb + (half2_t){q.y, -q.x}; }
        if (C == 1) { w1 = p - q; w2 = pb - (half2_t){q.y, -q.x}; }
        if (C == 2) { w1 = p + (half2_t){-q.y, q.x}; w2 = pb + (half2_t){q.x, q.y}; }
        if (C == 3) { w1 = p + (half2_t){q.y, -q.x}; w2 = pb + (half2_t){-q.x, -q.y}; }
    }
}

// a.x b.x + a.y b.y with exact binary16 products, FP32 result: the head of a dot
// product chain, written as the three-operand form with an inline zero (the
// compiler would otherwise start every chain with a register move of 0.0).
HD float dot2_first(uint32_t a, half2_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    float r;
    asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
    return r;
#else
    const half2_t x = as_h2(a);
    return (float)x.x * (float)b.x + (float)x.y * (float)b.y;
#endif
}

// a.x b.x + a.y b.y + c with exact binary16 products and FP32 accumulation
HD float dot2(uint32_t a, half2_t b, float c) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_fdot2(as_h2(a), b, c, false);
#else
    const half2_t x = as_h2(a);
    return (float)x.x * (float)b.x + (float)x.y * (float)b.y + c;
#endif
}

// acc += n * (e g)
template <int E> HD void recon16(float n, float gr, float gi, float& ar, float& ai) {
    if (E == 0) { ar = __builtin_fmaf(n, gr, ar); ai = __builtin_fmaf(n, gi, ai); }
    if (E == 1) { ar = __builtin_fmaf(-n, gr, ar); ai = __builtin_fmaf(-n, gi, ai); }
    if (E == 2) { ar = __builtin_fmaf(-n, gi, ar); ai = __builtin_fmaf(n, gr, ai); }
    if (E == 3) { ar = __builtin_fmaf(n, gi, ar); ai = __builtin_fmaf(-n, gr, ai); }
}

// One hopping term on raw words: acc += n (1 -/+ g_mu) U' psi, U' = U (forward) or
// U^dag (backward); w[spin*3 + colour] are the neighbour's words, u[a*3 + b] the link's.
template <int MU, bool FWD, bool G5IN, bool G5OUT>
HD void hop_term16(const uint32_t u[9], const uint32_t w[12], float n, float acc[24]) {
    using S = Spin<MU>;
    constexpr int fc = (FWD ? 0 : 1) ^ (G5IN ? 1 : 0);
    constexpr int fe = (FWD ? 0 : 1) ^ (G5OUT ? 1 : 0);
    half2_t w1[2][3], w2[2][3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        proj_h2<S::C0 ^ fc, FWD>(w[0 * 3 + b], w[S::Q0 * 3 + b], w1[0][b], w2[0][b]);
        proj_h2<S::C1 ^ fc, FWD>(w[1 * 3 + b], w[S::Q1 * 3 + b], w1[1][b], w2[1][b]);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const uint32_t l0 = FWD ? u[a * 3] : u[a];
            float gr = dot2_first(l0, w1[s][0]), gi = dot2_first(l0, w2[s][0]);
#pragma unroll
            for (int b = 1; b < 3; ++b) {
                const uint32_t l = FWD ? u[a * 3 + b] : u[b * 3 + a];
                gr = dot2(l, w1[s][b], gr);
                gi = dot2(l, w2[s][b], gi);
            }
            // upper spin s gets g_s; lower spins take theirs from the table
            acc[2 * (s * 3 + a)] = __builtin_fmaf(n, gr, acc[2 * (s * 3 + a)]);
            acc[2 * (s * 3 + a) + 1] = __builtin_fmaf(n, gi, acc[2 * (s * 3 + a) + 1]);
            if (S::R2 == s) recon16<S::E2 ^ fe>(n, gr, gi, acc[2 * (2 * 3 + a)], acc[2 * (2 * 3 + a) + 1]);
            if (S::R3 == s) recon16<S::E3 ^ fe>(n, gr, gi, acc[2 * (3 * 3 + a)], acc[2 * (3 * 3 + a) + 1]);
        }
}

// ---------------------------------------------------------------- clover block

// y = C x for one packed Hermitian 6x6 block held as 18 words (3 diagonal pairs,
// then the 15 lower entries), x given by an accessor returning FP32 values.
template <class X> HD void herm6_16(const uint32_t c[18], const X& x, float y[12]) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const uint32_t dw = c[i >> 1];
        const float d = (i & 1) ? hi16(dw) : lo16(dw);
        y[2 * i] = x.mul(d, 2 * i);
        y[2 * i + 1] = x.mul(d, 2 * i + 1);
    }
    int k = 0;
#pragma unroll
    for (int i = 1; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < i; ++j, ++k) {
            const uint32_t l = c[3 + k];
            y[2 * i] = x.fma(lo16(l), 2 * j, y[2 * i]);
            y[2 * i] = x.fma(-hi16(l), 2 * j + 1, y[2 * i]);
            y[2 * i + 1] = x.fma(lo16(l), 2 * j + 1, y[2 * i + 1]);
            y[2 * i + 1] = x.fma(hi16(l), 2 * j, y[2 * i + 1]);
            y[2 * j] = x.fma(lo16(l), 2 * i, y[2 * j]);
            y[2 * j] = x.fma(hi16(l), 2 * i + 1, y[2 * j]);
            y[2 * j + 1] = x.fma(lo16(l), 2 * i + 1, y[2 * j + 1]);
            y[2 * j + 1] = x.fma(-hi16(l), 2 * i, y[2 * j + 1]);
        }
}

// x as FP32 registers
struct XF {
    const float* v;
    HD float mul(float c, int i) const { return __builtin_fmaf(c, v[i], 0.f); }
    HD float fma(float c, int i, float y) const { return __builtin_fmaf(c, v[i], y); }
};
// x as six binary16 words (unscaled)
struct XW {
    const uint32_t* w;
    HD float val(int i) const { return (i & 1) ? hi16(w[i >> 1]) : lo16(w[i >> 1]); }
    HD float mul(float c, int i) const { return __builtin_fmaf(c, val(i), 0.f); }
    HD float fma(float c, int i, float y) const { return __builtin_fmaf(c, val(i), y); }
};

// The 18 words of one clover block (layout [block][5][Vh][4], the fifth group padded):
// site16 = 16 site, G16 = 16 Vh.
HD void load_clover16(const WSrc& C, uint32_t G16, int blk, uint32_t site16, uint32_t c[20]) {
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const u32x4 v = wld4(C, site16, (uint32_t)(blk * 5 + q) * G16);
        c[4 * q] = v.x; c[4 * q + 1] = v.y; c[4 * q + 2] = v.z; c[4 * q + 3] = v.w;
    }
}

// ---------------------------------------------------------------- spinor store

// Stores 24 FP32 values as binary16 words scaled by their largest magnitude
// (the rule of store_spinor in common.h) and returns the sum of their squares;
// the stored words and scale are left in w and m (the stored value is w * m).
HD float store16w(const F16Field& f, uint32_t G16, uint32_t site, const float s[24], uint32_t w[12], float& m) {
    m = 0.f;
#pragma unroll
    for (int i = 0; i < 24; ++i) m = fmaxf(m, fabsf(s[i]));
    if (!(m >= 1e-30f)) m = 0.f;
    const float inv = m > 0.f ? 1.0f / m : 0.f;
    wst(f.n, 4u * site, 0, __builtin_bit_cast(uint32_t, m));
    float q = 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        w[c] = f_to_h(s[2 * c] * inv) | (f_to_h(s[2 * c + 1] * inv) << 16);
        q = __builtin_fmaf(s[2 * c], s[2 * c], q);
        q = __builtin_fmaf(s[2 * c + 1], s[2 * c + 1], q);
    }
    wide_store_begin();
#pragma unroll
    for (int g = 0; g < 3; ++g) wst4(f.v, 16u * site, (uint32_t)g * G16, (u32x4){w[4 * g], w[4 * g + 1], w[4 * g + 2], w[4 * g + 3]});
    wide_store_end();
    return q;
}

HD float store16(const F16Field& f, uint32_t G16, uint32_t site, const float s[24]) {
    uint32_t w[12];
    float m;
    return store16w(f, G16, site, s, w, m);
}

// sum conj(a) b over the 12 complex components of two stored sites (binary16 words;
// the caller multiplies by both scales): exact binary16 products, FP32 sums, as
// v_dot2: re = ar br + ai bi, im = ar bi - ai br = (ar, ai) . (bi, -br)
HD void dot16(const uint32_t a[12], const uint32_t b[12], float& re, float& im) {
    re = 0.f;
    im = 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const half2_t bb = as_h2(b[c]);
        re = dot2(a[c], bb, re);
        im = dot2(a[c], (half2_t){bb.y, -bb.x}, im);
    }
}

// ---------------------------------------------------------------- LDS window

// The +-x and +-y neighbours of a block's sites lie within one y row of the block's
// own site range on the same timeslice (except across the periodic y boundary).
// The block copies that window of the input field into LDS once, with loads that
// write LDS directly (no registers), and takes those four neighbours from there:
// each input word then crosses the L1 data path, which bounds this stencil, about
// 5 times per use instead of 8.  Sites: w0 .. w0 + wn - 1 (clamped to the timeslice
// [lo, hi) when loaded: entries outside it are never read).  Layout per
// right-hand side j: word groups g = 0..2 as planes of wn 16-byte entries at word
// ((j*3 + g)*wn)*4, then the scales as planes of wn words at NB*12*wn + j*wn.
#if defined(__HIP_DEVICE_COMPILE__)
typedef __attribute__((address_space(3))) uint32_t* LdsWords;
typedef __attribute__((address_space(3))) const u32x4* LdsQuads;
#else
typedef uint32_t* LdsWords;
typedef const u32x4* LdsQuads;
#endif
struct Window16 {
    int wn, w0, lo, hi;
    LdsWords lds;
};

// Issues the window's loads for every right-hand side in use; the caller waits for
// them (window_ready) before reading.  Each wave fills 64 consecutive entries of a
// plane per load: the LDS address of lane l is the wave's base + l times the load size.
template <int NB, int BS>
HD void stage_window16(const Window16& W, const F16Field (&in)[NB], const bool (&use)[NB], uint32_t G16) {
#if defined(__HIP_DEVICE_COMPILE__)
    const int lane = (int)threadIdx.x & 63;
    for (int e0 = wave_uniform((int)threadIdx.x & ~63); e0 < W.wn; e0 += BS) {
        const int e = e0 + lane;
        if (e < W.wn) {
            int site = W.w0 + e;
            site = site < W.lo ? W.lo : (site >= W.hi ? W.hi - 1 : site);
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (use[j]) {
#pragma unroll
                    for (int g = 0; g < 3; ++g)
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(in[j].v.r, (__attribute__((address_space(3))) void*)(W.lds + ((j * 3 + g) * W.wn + e0) * 4),
                                                                 16, 16 * site, g * (int)G16, 0, 0);
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(in[j].n.r, (__attribute__((address_space(3))) void*)(W.lds + NB * 12 * W.wn + j * W.wn + e0),
                                                             4, 4 * site, 0, 0, 0);
                }
        }
    }
#else
    (void)W; (void)in; (void)use; (void)G16;
#endif
}

// Makes the window visible to the block: every wave waits for its own LDS loads,
// then the block meets.
HD void window_ready() {
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); other counters unconstrained
    __syncthreads();
#endif
}

// Words and scale of neighbour site nsite of right-hand side j: from the window
// when the site lies in it, else from the field.
template <int NB>
HD float window_words(const Window16& W, const F16Field& f, int j, uint32_t nsite, uint32_t G16, uint32_t w[12]) {
    const uint32_t i = nsite - (uint32_t)W.w0;
    const bool inw = i < (uint32_t)W.wn;
    float n = 0.f;
    if (W.wn > 0) {
        const uint32_t li = inw ? i : 0u;
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            const u32x4 v = ((LdsQuads)W.lds)[(uint32_t)((j * 3 + g) * W.wn) + li];
            w[4 * g] = v.x; w[4 * g + 1] = v.y; w[4 * g + 2] = v.z; w[4 * g + 3] = v.w;
        }
        n = __builtin_bit_cast(float, W.lds[(uint32_t)(NB * 12 * W.wn + j * W.wn) + li]);
    }
    if (!inw) {
        load_words(f, 16u * nsite, G16, w);
        n = wldf(f.n, 4u * nsite, 0);
    }
    return n;
}

// ---------------------------------------------------------------- site body

// Both hops in direction MU; WIN: the neighbours come through the LDS window.
template <int NB, int MU, bool G5IN, bool G5OUT, bool WIN>
HD void hop_dir16(const HopJob<P16>& J, const WSrc& U, const F16Field (&in)[NB], const Nbr& nb, uint32_t site,
                  const bool (&use)[NB], const float (&sc)[NB], const Window16& W, float (&acc)[NB][24]) {
    const uint32_t Vh = (uint32_t)J.g.Vh;
    uint32_t u[9], w[NB][12];
    float n[NB];
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        const uint32_t ns = (uint32_t)nb.n[2 * MU + d];
        // forward hop: the link of this site; backward: the neighbour's, of the other parity
        load_link16(U, 12u * (d == 0 ? site : ns), 12u * Vh, d == 0 ? J.par : 1 - J.par, MU, u);
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (use[j]) {
                if (WIN) {
                    n[j] = window_words<NB>(W, in[j], j, ns, 16u * Vh, w[j]);
                } else {
                    load_words(in[j], 16u * ns, 16u * Vh, w[j]);
                    n[j] = wldf(in[j].n, 4u * ns, 0);
                }
            }
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (use[j]) {
                if (d == 0) hop_term16<MU, true, G5IN, G5OUT>(u, w[j], n[j] * sc[j], acc[j]);
                else hop_term16<MU, false, G5IN, G5OUT>(u, w[j], n[j] * sc[j], acc[j]);
            }
    }
}

// out = ... as in hop_site (hop.h) for P16 fields; the partial-sum contributions qs
// as there.  Every thread of the block calls it (W's staging has a block barrier); a
// thread with !valid works on a real site but stores nothing and returns qs = 0.
template <int NB, int KIND, int FL, int BS>
HD void hop_site16(const HopJob<P16>& J, int cb, int g0, bool valid, const Window16& W, double (&qs)[NB][HOP_NQ_MAX]) {
    const uint32_t G16 = 16u * (uint32_t)J.g.Vh;  // bytes per 16-byte group plane
    const uint32_t site = (uint32_t)cb, lo = 4u * site, s16 = 16u * site;
    constexpr bool G5IN = (FL & F_G5IN) != 0;
    constexpr bool G5OUT = (FL & F_G5OUT) != 0;
    constexpr bool CG = (KIND == K2) && (FL & F_CG);
    bool use[NB];
    float sc[NB], al[NB];
    F16Field in[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int r = g0 + j;
        use[j] = rhs_active(J, r);
        for (int q = 0; q < HOP_NQ_MAX; ++q) qs[j][q] = 0.0;
        in[j] = f16_field(J.in, J.g.Vh, r);
        al[j] = CG ? (float)J.alpha[r < J.nrhs ? r : 0] : 0.f;
        // K2 with the CG update accumulates -alpha * out directly
        sc[j] = CG ? (float)(-J.ch) * al[j] : (float)J.ch;
    }
    float acc[NB][24];
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int i = 0; i < 24; ++i) acc[j][i] = 0.f;

    const WSrc U = wsrc(J.U, 288u * (uint32_t)J.g.Vh);
    const Nbr nb = neighbours(J.g, J.par, cb);
    // the window's loads fly while the t and z hops run on loads of their own
    if (W.wn > 0) stage_window16<NB, BS>(W, in, use, G16);
    hop_dir16<NB, 0, G5IN, G5OUT, false>(J, U, in, nb, site, use, sc, W, acc);
    hop_dir16<NB, 3, G5IN, G5OUT, false>(J, U, in, nb, site, use, sc, W, acc);
    if (W.wn > 0) window_ready();
    hop_dir16<NB, 1, G5IN, G5OUT, true>(J, U, in, nb, site, use, sc, W, acc);
    hop_dir16<NB, 2, G5IN, G5OUT, true>(J, U, in, nb, site, use, sc, W, acc);

    const WSrc C = wsrc(J.C, 10u * G16);
    if (KIND == K1) {
        if (FL & F_HASD) {
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (use[j]) {
                    const F16Field d = f16_field(J.x, J.g.Vh, g0 + j);
                    const float n = wldf<CP_NT>(d.n, lo, 0);
                    uint32_t ow[12];
                    load_words<CP_NT>(d, s16, G16, ow);
#pragma unroll
                    for (int c = 0; c < 12; ++c) {
                        const uint32_t w = ow[c];
                        acc[j][2 * c] = __builtin_fmaf(lo16(w), n, acc[j][2 * c]);
                        acc[j][2 * c + 1] = __builtin_fmaf(hi16(w), n, acc[j][2 * c + 1]);
                    }
                }
        }
#pragma unroll
        for (int blk = 0; blk < 2; ++blk) {
            uint32_t c[20];
            load_clover16(C, G16, blk, s16, c);
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (use[j]) {
                    float t[12];
                    herm6_16(c, XF{&acc[j][blk * 12]}, t);
#pragma unroll
                    for (int i = 0; i < 12; ++i) acc[j][blk * 12 + i] = t[i];
                }
        }
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (use[j]) {
                const F16Field o = f16_field(J.out, J.g.Vh, g0 + j);
                if (FL & F_ACCUM) {
                    const float n = wldf<CP_NT>(o.n, lo, 0);
                    uint32_t ow[12];
                    load_words<CP_NT>(o, s16, G16, ow);
#pragma unroll
                    for (int c = 0; c < 12; ++c) {
                        const uint32_t w = ow[c];
                        acc[j][2 * c] = __builtin_fmaf(lo16(w), n, acc[j][2 * c]);
                        acc[j][2 * c + 1] = __builtin_fmaf(hi16(w), n, acc[j][2 * c + 1]);
                    }
                }
                if (valid) {
                    const float q = store16(o, G16, site, acc[j]);
                    if (FL & F_NORM) qs[j][0] = (double)q;
                }
            }
    } else {
        // clover (or identity) term on x: acc += ca' * n_x * (A x^)
        uint32_t xw[NB][12];
        float nx[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (use[j]) {
                const F16Field xf = f16_field(J.x, J.g.Vh, g0 + j);
                nx[j] = wldf<CP_NT>(xf.n, lo, 0);
                load_words<CP_NT>(xf, s16, G16, xw[j]);
            }
#pragma unroll
        for (int blk = 0; blk < 2; ++blk) {
            uint32_t c[20];
            if (!(FL & F_NOA)) load_clover16(C, G16, blk, s16, c);
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (use[j]) {
                    const float f = (CG ? -(float)J.ca * al[j] : (float)J.ca) * nx[j];
                    if (FL & F_NOA) {
#pragma unroll
                        for (int i = 0; i < 6; ++i) {
                            const uint32_t w = xw[j][blk * 6 + i];
                            acc[j][blk * 12 + 2 * i] = __builtin_fmaf(lo16(w), f, acc[j][blk * 12 + 2 * i]);
                            acc[j][blk * 12 + 2 * i + 1] = __builtin_fmaf(hi16(w), f, acc[j][blk * 12 + 2 * i + 1]);
                        }
                    } else {
                        float t[12];
                        herm6_16(c, XW{&xw[j][blk * 6]}, t);
#pragma unroll
                        for (int i = 0; i < 12; ++i) acc[j][blk * 12 + i] = __builtin_fmaf(f, t[i], acc[j][blk * 12 + i]);
                    }
                }
        }
        // F_DOTR: r is the shadow residual, one field for every right-hand side (its view
        // has RHS stride 0): loaded once per site, not once per right-hand side.  (With
        // F_DOTXH the same hoisting pushes the kernel past its register budget.)
        uint32_t rw[12];
        float nr = 0.f;
        if (FL & F_DOTR) {
            const F16Field rf = f16_field(J.r, J.g.Vh, 0);
            nr = wldf(rf.n, lo, 0);  // cached: one field for every RHS
            load_words(rf, s16, G16, rw);
        }
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (use[j]) {
                if (FL & F_HASB) {
                    const F16Field bf = f16_field(J.b, J.g.Vh, g0 + j);
                    const float n = wldf<CP_NT>(bf.n, lo, 0) * (float)J.cb;
                    uint32_t ow[12];
                    load_words<CP_NT>(bf, s16, G16, ow);
#pragma unroll
                    for (int c = 0; c < 12; ++c) {
                        const uint32_t w = ow[c];
                        acc[j][2 * c] = __builtin_fmaf(lo16(w), n, acc[j][2 * c]);
                        acc[j][2 * c + 1] = __builtin_fmaf(hi16(w), n, acc[j][2 * c + 1]);
                    }
                }
                if (CG) {
                    // r -= alpha out  (acc already holds -alpha out)
                    const F16Field rf = f16_field(J.r, J.g.Vh, g0 + j);
                    const float nr = wldf<CP_NT>(rf.n, lo, 0);
                    uint32_t ow[12];
                    load_words<CP_NT>(rf, s16, G16, ow);
#pragma unroll
                    for (int c = 0; c < 12; ++c) {
                        const uint32_t w = ow[c];
                        acc[j][2 * c] = __builtin_fmaf(lo16(w), nr, acc[j][2 * c]);
                        acc[j][2 * c + 1] = __builtin_fmaf(hi16(w), nr, acc[j][2 * c + 1]);
                    }
                    if (valid) qs[j][0] = (double)store16(rf, G16, site, acc[j]);
                    // xs += alpha x
                    const F16Field sf = f16_field(J.xs, J.g.Vh, g0 + j);
                    const float ns = wldf<CP_NT>(sf.n, lo, 0), ax = al[j] * nx[j];
                    load_words<CP_NT>(sf, s16, G16, ow);
#pragma unroll
                    for (int c = 0; c < 12; ++c) {
                        const uint32_t w = ow[c];
                        acc[j][2 * c] = __builtin_fmaf(lo16(xw[j][c]), ax, __builtin_fmaf(lo16(w), ns, 0.f));
                        acc[j][2 * c + 1] = __builtin_fmaf(hi16(xw[j][c]), ax, __builtin_fmaf(hi16(w), ns, 0.f));
                    }
                    if (valid) (void)store16(sf, G16, site, acc[j]);
                } else if (valid) {
                    const F16Field o = f16_field(J.out, J.g.Vh, g0 + j);
                    uint32_t ow[12];
                    float om;
                    const float q = store16w(o, G16, site, acc[j], ow, om);
                    if (FL & F_NORM) qs[j][0] = (double)q;
                    if (FL & F_DOTX) {  // sum conj(out) x, with x's words and scale in registers
                        float re = 0.f, im = 0.f;
#pragma unroll
                        for (int c = 0; c < 12; ++c) {
                            const float xr = lo16(xw[j][c]), xi = hi16(xw[j][c]);
                            re = __builtin_fmaf(acc[j][2 * c], xr, __builtin_fmaf(acc[j][2 * c + 1], xi, re));
                            im = __builtin_fmaf(acc[j][2 * c], xi, __builtin_fmaf(-acc[j][2 * c + 1], xr, im));
                        }
                        qs[j][0] = (double)re * nx[j];
                        qs[j][1] = (double)im * nx[j];
                        qs[j][2] = (double)q;
                    }
                    if (FL & F_DOTXH) {  // sum conj(r) out of the stored out, r (the shadow residual) at the own site
                        const F16Field rf = f16_field(J.r, J.g.Vh, g0 + j);
                        const float nrh = wldf(rf.n, lo, 0);  // cached: one field for every RHS
                        uint32_t rwh[12];
                        load_words(rf, s16, G16, rwh);
                        float re, im;
                        dot16(rwh, ow, re, im);
                        qs[j][3] = (double)re * ((double)nrh * om);
                        qs[j][4] = (double)im * ((double)nrh * om);
                    }
                    if (FL & F_DOTR) {  // sum conj(r) out, r (the shadow residual) at the own site
                        float re = 0.f, im = 0.f;
#pragma unroll
                        for (int c = 0; c < 12; ++c) {
                            const float rr = lo16(rw[c]), ri = hi16(rw[c]);
                            re = __builtin_fmaf(rr, acc[j][2 * c], __builtin_fmaf(ri, acc[j][2 * c + 1], re));
                            im = __builtin_fmaf(rr, acc[j][2 * c + 1], __builtin_fmaf(-ri, acc[j][2 * c], im));
                        }
                        qs[j][0] = (double)re * nr;
                        qs[j][1] = (double)im * nr;
                    }
                }
            }
    }
}

}  // namespace dlma
