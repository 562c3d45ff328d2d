// Wilson hop terms with spin projection, and link/spinor loads from the
// native layouts. Shared by the stencil and the Schwarz block kernels.
//
// With g_mu = [[0, e_mu], [e_mu^+, 0]] (e_0 = -1, e_k = -i sigma_k) and e_mu
// unitary, (1 - g_mu) psi = [h; -e_mu^+ h] with h = psi_up - e_mu psi_lo, and
// (1 + g_mu) psi = [k; e_mu^+ k] with k = psi_up + e_mu psi_lo. A hop thus
// multiplies two colour vectors by the link instead of four.
#pragma once

#include "internal.h"

namespace dfl {

__device__ inline float bf16_to_f(uint32_t bits16) { return __uint_as_float(bits16 << 16); }

// Loads take a uniform base and a 32-bit byte offset (see toff).
template <typename E> __device__ inline E ld(const E* __restrict__ plane, uint32_t byte_off)
{
    return *reinterpret_cast<const E*>(reinterpret_cast<const char*>(plane) + byte_off);
}
template <typename E> __device__ inline void st(E* __restrict__ plane, uint32_t byte_off, E v)
{
    *reinterpret_cast<E*>(reinterpret_cast<char*>(plane) + byte_off) = v;
}

// byte offset of entry c (of ncomp per site) of site s; fits 32 bits because
// fields hold fewer than 2^24 sites (checked at context creation)
template <typename E> __device__ inline uint32_t toff(long s, int c, int ncomp)
{
    return (uint32_t)tidx(s, c, ncomp) * (uint32_t)sizeof(E);
}

__device__ inline su3<double> load_link(const Links64& L, int mu, long s)
{
    su3<double> u;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            u.m[a][b] = ld(L.u, toff<c64>(s, mu * 6 + a * 3 + b, 24));
    complete_third_row(u);
    return u;
}

__device__ inline su3<float> load_link(const Links32& L, int mu, long s)
{
    su3<float> u;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            u.m[a][b] = ld(L.u, toff<c32>(s, mu * 6 + a * 3 + b, 24));
    complete_third_row(u);
    return u;
}

__device__ inline su3<float> load_link(const LinksBF16& L, int mu, long s)
{
    su3<float> u;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            uint32_t w = ld(L.u, toff<uint32_t>(s, mu * 6 + a * 3 + b, 24));
            u.m[a][b] = c32{bf16_to_f(w & 0xffffu), bf16_to_f(w >> 16)};
        }
    complete_third_row(u);
    return u;
}

// The two stored rows of a link, loaded ahead of their use (the third row is
// completed only when the matrix is needed, so that a load in flight holds 12
// instead of 18 values).
template <typename L> struct LinkRows;
template <> struct LinkRows<Links64> {
    c64 e[6];
};
template <> struct LinkRows<Links32> {
    c32 e[6];
};
template <> struct LinkRows<LinksBF16> {
    uint32_t e[6];
};
__device__ inline LinkRows<Links64> load_rows(const Links64& L, int mu, long s)
{
    LinkRows<Links64> r;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        r.e[q] = ld(L.u, toff<c64>(s, mu * 6 + q, 24));
    return r;
}
__device__ inline LinkRows<Links32> load_rows(const Links32& L, int mu, long s)
{
    LinkRows<Links32> r;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        r.e[q] = ld(L.u, toff<c32>(s, mu * 6 + q, 24));
    return r;
}
__device__ inline LinkRows<LinksBF16> load_rows(const LinksBF16& L, int mu, long s)
{
    LinkRows<LinksBF16> r;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        r.e[q] = ld(L.u, toff<uint32_t>(s, mu * 6 + q, 24));
    return r;
}
__device__ inline su3<double> to_link(const LinkRows<Links64>& r)
{
    su3<double> u;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        u.m[q / 3][q % 3] = r.e[q];
    complete_third_row(u);
    return u;
}
__device__ inline su3<float> to_link(const LinkRows<Links32>& r)
{
    su3<float> u;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        u.m[q / 3][q % 3] = r.e[q];
    complete_third_row(u);
    return u;
}
__device__ inline su3<float> to_link(const LinkRows<LinksBF16>& r)
{
    su3<float> u;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        u.m[q / 3][q % 3] = c32{bf16_to_f(r.e[q] & 0xffffu), bf16_to_f(r.e[q] >> 16)};
    complete_third_row(u);
    return u;
}

template <typename T> __device__ inline spinor<T> load_spinor(const cpx<T>* __restrict__ f, long V, long s)
{
    (void)V;
    spinor<T> p;
#pragma unroll
    for (int al = 0; al < 4; ++al)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            p.s[al].c[a] = ld(f, toff<cpx<T>>(s, 3 * al + a, 12));
    return p;
}

template <typename T> __device__ inline void store_spinor(cpx<T>* __restrict__ f, long V, long s, const spinor<T>& p)
{
    (void)V;
#pragma unroll
    for (int al = 0; al < 4; ++al)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            st(f, toff<cpx<T>>(s, 3 * al + a, 12), p.s[al].c[a]);
}

template <typename T> __device__ inline void zero(spinor<T>& p)
{
#pragma unroll
    for (int al = 0; al < 4; ++al)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            p.s[al].c[a] = cpx<T>{0, 0};
}

// The spin projections of the two hops: (1 - g_mu) psi = [h0, h1; ...] for the
// forward hop and (1 + g_mu) psi = [k0, k1; ...] for the backward one; the
// lower two spin components follow from the upper ones (fwd_add, bwd_add).
template <int MU, typename T> __device__ inline void proj_fwd(const spinor<T>& p, cvec3<T>& h0, cvec3<T>& h1)
{
    if (MU == 0) {
        h0 = p.s[0] + p.s[2];
        h1 = p.s[1] + p.s[3];
    } else if (MU == 1) {
        h0 = p.s[0] + vi(p.s[3]);
        h1 = p.s[1] + vi(p.s[2]);
    } else if (MU == 2) {
        h0 = p.s[0] + p.s[3];
        h1 = p.s[1] - p.s[2];
    } else {
        h0 = p.s[0] + vi(p.s[2]);
        h1 = p.s[1] - vi(p.s[3]);
    }
}
template <int MU, typename T> __device__ inline void proj_bwd(const spinor<T>& p, cvec3<T>& k0, cvec3<T>& k1)
{
    if (MU == 0) {
        k0 = p.s[0] - p.s[2];
        k1 = p.s[1] - p.s[3];
    } else if (MU == 1) {
        k0 = p.s[0] + vmi(p.s[3]);
        k1 = p.s[1] + vmi(p.s[2]);
    } else if (MU == 2) {
        k0 = p.s[0] - p.s[3];
        k1 = p.s[1] + p.s[2];
    } else {
        k0 = p.s[0] + vmi(p.s[2]);
        k1 = p.s[1] + vi(p.s[3]);
    }
}

// acc += the four spin components of (1 - g_mu) U psi_fwd from u0 = U h0, u1 = U h1
template <int MU, typename T> __device__ inline void fwd_add(const cvec3<T>& u0, const cvec3<T>& u1, spinor<T>& acc)
{
    acc.s[0] += u0;
    acc.s[1] += u1;
    if (MU == 0) {
        acc.s[2] += u0;
        acc.s[3] += u1;
    } else if (MU == 1) {
        acc.s[2] += vmi(u1);
        acc.s[3] += vmi(u0);
    } else if (MU == 2) {
        acc.s[2] -= u1;
        acc.s[3] += u0;
    } else {
        acc.s[2] += vmi(u0);
        acc.s[3] += vi(u1);
    }
}

// acc += (1 - g_mu) U psi_fwd
template <int MU, typename T>
__device__ inline void hop_fwd(const su3<T>& u, const spinor<T>& p, spinor<T>& acc)
{
    cvec3<T> h0, h1;
    proj_fwd<MU>(p, h0, h1);
    fwd_add<MU>(mul(u, h0), mul(u, h1), acc);
}

// The backward hop in two halves: the spin-projected colour vectors
// v = U^+ k of (1 + g_mu) U^+ psi_bwd, and their reconstruction into the four
// spin components (bwd_add).
template <int MU, typename T>
__device__ inline void bwd_project(const su3<T>& u, const spinor<T>& p, cvec3<T>& v0, cvec3<T>& v1)
{
    cvec3<T> k0, k1;
    proj_bwd<MU>(p, k0, k1);
    v0 = mul_dag(u, k0);
    v1 = mul_dag(u, k1);
}

template <int MU, typename T> __device__ inline void bwd_add(const cvec3<T>& v0, const cvec3<T>& v1, spinor<T>& acc)
{
    acc.s[0] += v0;
    acc.s[1] += v1;
    if (MU == 0) {
        acc.s[2] -= v0;
        acc.s[3] -= v1;
    } else if (MU == 1) {
        acc.s[2] += vi(v1);
        acc.s[3] += vi(v0);
    } else if (MU == 2) {
        acc.s[2] += v1;
        acc.s[3] -= v0;
    } else {
        acc.s[2] += vi(v0);
        acc.s[3] += vmi(v1);
    }
}

// acc += (1 + g_mu) U^+ psi_bwd   (u is the link U_mu(x - mu))
template <int MU, typename T>
__device__ inline void hop_bwd(const su3<T>& u, const spinor<T>& p, spinor<T>& acc)
{
    cvec3<T> v0, v1;
    bwd_project<MU>(u, p, v0, v1);
    bwd_add<MU>(v0, v1, acc);
}

// runtime-direction forms (uniform branch on mu)
template <typename T>
__device__ inline void hop_fwd_rt(int mu, const su3<T>& u, const spinor<T>& p, spinor<T>& acc)
{
    switch (mu) {
    case 0: hop_fwd<0>(u, p, acc); break;
    case 1: hop_fwd<1>(u, p, acc); break;
    case 2: hop_fwd<2>(u, p, acc); break;
    default: hop_fwd<3>(u, p, acc); break;
    }
}
template <typename T>
__device__ inline void hop_bwd_rt(int mu, const su3<T>& u, const spinor<T>& p, spinor<T>& acc)
{
    switch (mu) {
    case 0: hop_bwd<0>(u, p, acc); break;
    case 1: hop_bwd<1>(u, p, acc); break;
    case 2: hop_bwd<2>(u, p, acc); break;
    default: hop_bwd<3>(u, p, acc); break;
    }
}

// runtime-direction projection (a = h0 or k0, b = h1 or k1) and accumulation
// of the projected neighbour multiplied by the link (U for step > 0, U^+ for
// step < 0)
template <typename T>
__device__ inline void proj_rt(int mu, int step, const spinor<T>& p, cvec3<T>& a, cvec3<T>& b)
{
    if (step > 0) {
        switch (mu) {
        case 0: proj_fwd<0>(p, a, b); break;
        case 1: proj_fwd<1>(p, a, b); break;
        case 2: proj_fwd<2>(p, a, b); break;
        default: proj_fwd<3>(p, a, b); break;
        }
    } else {
        switch (mu) {
        case 0: proj_bwd<0>(p, a, b); break;
        case 1: proj_bwd<1>(p, a, b); break;
        case 2: proj_bwd<2>(p, a, b); break;
        default: proj_bwd<3>(p, a, b); break;
        }
    }
}
template <int MU, int STEP, typename T>
__device__ inline void hop_add(const su3<T>& u, const cvec3<T>& a, const cvec3<T>& b, spinor<T>& acc)
{
    if (STEP > 0)
        fwd_add<MU>(mul(u, a), mul(u, b), acc);
    else
        bwd_add<MU>(mul_dag(u, a), mul_dag(u, b), acc);
}
template <typename T>
__device__ inline void hop_add_rt(int mu, int step, const su3<T>& u, const cvec3<T>& a, const cvec3<T>& b,
                                  spinor<T>& acc)
{
    if (step > 0) {
        switch (mu) {
        case 0: hop_add<0, 1>(u, a, b, acc); break;
        case 1: hop_add<1, 1>(u, a, b, acc); break;
        case 2: hop_add<2, 1>(u, a, b, acc); break;
        default: hop_add<3, 1>(u, a, b, acc); break;
        }
    } else {
        switch (mu) {
        case 0: hop_add<0, -1>(u, a, b, acc); break;
        case 1: hop_add<1, -1>(u, a, b, acc); break;
        case 2: hop_add<2, -1>(u, a, b, acc); break;
        default: hop_add<3, -1>(u, a, b, acc); break;
        }
    }
}

// -p (the neighbour of a hop across the time boundary of an antiperiodic field)
template <typename T> __device__ inline void negate(spinor<T>& p)
{
#pragma unroll
    for (int al = 0; al < 4; ++al)
        p.s[al] = cvec3<T>{{-p.s[al].c[0], -p.s[al].c[1], -p.s[al].c[2]}};
}

// The clover term of the O(a)-improved operator (section 2.1): per site a
// hermitian 12 x 12 matrix that commutes with gamma_5, i.e. two hermitian
// 6 x 6 blocks, one per chirality (spins 0, 1 and spins 2, 3; index
// 3 * (spin % 2) + colour inside a block). Each block is stored as 18 complex
// entries: slots 0..2 hold the six real diagonal entries as (d0, d1), (d2, d3),
// (d4, d5), slots 3..17 the entries (i, j), i < j, row by row. 36 entries per
// site in the 64-site tiling (kCloverComp). c == nullptr: no clover term.
template <typename T> struct Clover {
    const cpx<T>* c;
};

// o += C(x) p for site s
template <typename T> __device__ inline void clover_add(const Clover<T>& C, long s, const spinor<T>& p, spinor<T>& o)
{
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        cpx<T> e[18];
#pragma unroll
        for (int q = 0; q < 18; ++q)
            e[q] = ld(C.c, toff<cpx<T>>(s, 18 * h + q, kCloverComp));
        cpx<T> v[6], w[6];
#pragma unroll
        for (int i = 0; i < 6; ++i)
            v[i] = p.s[2 * h + i / 3].c[i % 3];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const T d = (i & 1) ? e[i / 2].im : e[i / 2].re;
            w[i] = cpx<T>{d * v[i].re, d * v[i].im};
        }
        int q = 3;
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = i + 1; j < 6; ++j, ++q) {
                w[i] += e[q] * v[j];               // C_ij v_j
                w[j] += cmul_conj(e[q], v[i]);     // C_ji v_i = conj(C_ij) v_i
            }
#pragma unroll
        for (int i = 0; i < 6; ++i)
            o.s[2 * h + i / 3].c[i % 3] += w[i];
    }
}

// out = diag * p - 1/2 acc
template <typename T>
__device__ inline spinor<T> finish(const spinor<T>& p, const spinor<T>& acc, T diag)
{
    spinor<T> o;
#pragma unroll
    for (int al = 0; al < 4; ++al)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            o.s[al].c[a].re = diag * p.s[al].c[a].re - T(0.5) * acc.s[al].c[a].re;
            o.s[al].c[a].im = diag * p.s[al].c[a].im - T(0.5) * acc.s[al].c[a].im;
        }
    return o;
}

}  // namespace dfl
