// Device-side building blocks shared by the HIP kernels of the solver:
// complex numbers, colour vectors and SU(3) links, the block-major native
// site layout, XCD-aware workgroup numbering and wavefront reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dfl {

// ------------------------------------------------------------ complex

template <typename T> struct alignas(2 * sizeof(T)) cpx {
    T re, im;
};

template <typename T> __host__ __device__ inline cpx<T> mk(T r, T i) { return cpx<T>{r, i}; }
template <typename T> __device__ inline cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __device__ inline cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __device__ inline cpx<T> operator-(cpx<T> a) { return {-a.re, -a.im}; }
template <typename T> __device__ inline cpx<T> operator*(cpx<T> a, cpx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __device__ inline cpx<T> operator*(T s, cpx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __device__ inline cpx<T>& operator+=(cpx<T>& a, cpx<T> b)
{
    a.re += b.re;
    a.im += b.im;
    return a;
}
template <typename T> __device__ inline cpx<T>& operator-=(cpx<T>& a, cpx<T> b)
{
    a.re -= b.re;
    a.im -= b.im;
    return a;
}
template <typename T> __device__ inline cpx<T> conjg(cpx<T> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename T> __device__ inline cpx<T> cmul_conj(cpx<T> a, cpx<T> b)
{
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// i * a and -i * a
template <typename T> __device__ inline cpx<T> times_i(cpx<T> a) { return {-a.im, a.re}; }
template <typename T> __device__ inline cpx<T> times_mi(cpx<T> a) { return {a.im, -a.re}; }

template <typename T> struct cvec3 {
    cpx<T> c[3];
};
template <typename T> __device__ inline cvec3<T> operator+(const cvec3<T>& a, const cvec3<T>& b)
{
    return {{a.c[0] + b.c[0], a.c[1] + b.c[1], a.c[2] + b.c[2]}};
}
template <typename T> __device__ inline cvec3<T> operator-(const cvec3<T>& a, const cvec3<T>& b)
{
    return {{a.c[0] - b.c[0], a.c[1] - b.c[1], a.c[2] - b.c[2]}};
}
template <typename T> __device__ inline cvec3<T> vi(const cvec3<T>& a)
{
    return {{times_i(a.c[0]), times_i(a.c[1]), times_i(a.c[2])}};
}
template <typename T> __device__ inline cvec3<T> vmi(const cvec3<T>& a)
{
    return {{times_mi(a.c[0]), times_mi(a.c[1]), times_mi(a.c[2])}};
}
template <typename T> __device__ inline void operator+=(cvec3<T>& a, const cvec3<T>& b)
{
    a.c[0] += b.c[0];
    a.c[1] += b.c[1];
    a.c[2] += b.c[2];
}
template <typename T> __device__ inline void operator-=(cvec3<T>& a, const cvec3<T>& b)
{
    a.c[0] -= b.c[0];
    a.c[1] -= b.c[1];
    a.c[2] -= b.c[2];
}

// SU(3) link as 3x3 complex, m[row][col]
template <typename T> struct su3 {
    cpx<T> m[3][3];
};

// U v
// fused multiply-add a * b + c (one rounding)
template <typename T> __device__ inline T fmadd(T a, T b, T c)
{
    if constexpr (sizeof(T) == sizeof(double))
        return __builtin_fma(a, b, c);
    else
        return __builtin_fmaf(a, b, c);
}

// c + a * b as four fused multiply-adds
template <typename T> __device__ inline cpx<T> cfma(cpx<T> a, cpx<T> b, cpx<T> c)
{
    return {fmadd(-a.im, b.im, fmadd(a.re, b.re, c.re)), fmadd(a.im, b.re, fmadd(a.re, b.im, c.im))};
}

// Row sums of three complex products as one chain of fused multiply-adds per
// real part (a sum of products written with complex operators compiles to a
// multiply, a multiply-add and an add per product and component instead).
template <typename T> __device__ inline cvec3<T> mul(const su3<T>& u, const cvec3<T>& v)
{
    cvec3<T> r;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T re = u.m[a][0].re * v.c[0].re, im = u.m[a][0].re * v.c[0].im;
        re = fmadd(-u.m[a][0].im, v.c[0].im, re);
        im = fmadd(u.m[a][0].im, v.c[0].re, im);
#pragma unroll
        for (int b = 1; b < 3; ++b) {
            re = fmadd(u.m[a][b].re, v.c[b].re, re);
            re = fmadd(-u.m[a][b].im, v.c[b].im, re);
            im = fmadd(u.m[a][b].re, v.c[b].im, im);
            im = fmadd(u.m[a][b].im, v.c[b].re, im);
        }
        r.c[a] = cpx<T>{re, im};
    }
    return r;
}
// U^dagger v
template <typename T> __device__ inline cvec3<T> mul_dag(const su3<T>& u, const cvec3<T>& v)
{
    cvec3<T> r;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T re = u.m[0][a].re * v.c[0].re, im = u.m[0][a].re * v.c[0].im;
        re = fmadd(u.m[0][a].im, v.c[0].im, re);
        im = fmadd(-u.m[0][a].im, v.c[0].re, im);
#pragma unroll
        for (int b = 1; b < 3; ++b) {
            re = fmadd(u.m[b][a].re, v.c[b].re, re);
            re = fmadd(u.m[b][a].im, v.c[b].im, re);
            im = fmadd(u.m[b][a].re, v.c[b].im, im);
            im = fmadd(-u.m[b][a].im, v.c[b].re, im);
        }
        r.c[a] = cpx<T>{re, im};
    }
    return r;
}
// third row of an SU(3) matrix from the first two: conj(row0 x row1)
template <typename T> __device__ inline void complete_third_row(su3<T>& u)
{
    // conj(a b - c d) with one fused chain per real part
    auto cross = [](cpx<T> a, cpx<T> b, cpx<T> c, cpx<T> d) {
        T re = a.re * b.re, im = a.re * b.im;
        re = fmadd(-a.im, b.im, re);
        im = fmadd(a.im, b.re, im);
        re = fmadd(-c.re, d.re, re);
        im = fmadd(-c.re, d.im, im);
        re = fmadd(c.im, d.im, re);
        im = fmadd(-c.im, d.re, im);
        return cpx<T>{re, -im};
    };
    u.m[2][0] = cross(u.m[0][1], u.m[1][2], u.m[0][2], u.m[1][1]);
    u.m[2][1] = cross(u.m[0][2], u.m[1][0], u.m[0][0], u.m[1][2]);
    u.m[2][2] = cross(u.m[0][0], u.m[1][1], u.m[0][1], u.m[1][0]);
}

// quark field value at one site: 4 spins x 3 colours
template <typename T> struct spinor {
    cvec3<T> s[4];
};

// ------------------------------------------------------------- layout
//
// Native quark field: sites are grouped in tiles of 64 (one wavefront); inside
// a tile the 12 components (c = 3*spin + colour) are stored one after the
// other, each as 64 consecutive complex values: element (s, c) at
// ((s / 64) * 12 + c) * 64 + s % 64. A wavefront's spinors are thus one
// contiguous 12 KB (FP64) run, and each component load is a 1 KB line.
// Links use the same tiling with 36 (FP64, 4 x 3 x 3) or 24 (two-row, 4 x 2 x 3)
// entries per site. Sites are numbered block-major over the deflation
// ("layout") blocks:
//   site = blk*Vb + ((y0*b1 + y1)*b2 + y2)*b3 + y3,
//   blk  = ((n0*nb1 + n1)*nb2 + n2)*nb3 + n3,
// with x_mu = n_mu*b_mu + y_mu. Every block is a contiguous run of Vb sites.

constexpr int kTile = 64;

// index of entry c (of ncomp per site) of site s in the tiled layout
__host__ __device__ inline long tidx(long s, int c, int ncomp)
{
    return ((s >> 6) * ncomp + c) * kTile + (s & (kTile - 1));
}

struct Geom {
    int L[4];     // lattice extent
    int b[4];     // layout block
    int nb[4];    // blocks per direction
    int lstr[4];  // in-block stride of y_mu
    int bstr[4];  // block-index stride of n_mu
    int Vb;       // sites per block
    int Nb;       // number of blocks
    long V;       // sites
    int tsign;    // quark boundary condition in direction 0: +1 periodic, -1 antiperiodic
};

__host__ inline Geom make_geom(const int L[4], const int b[4])
{
    Geom g;
    for (int mu = 0; mu < 4; ++mu) {
        g.L[mu] = L[mu];
        g.b[mu] = b[mu];
        g.nb[mu] = L[mu] / b[mu];
    }
    g.lstr[3] = 1;
    g.bstr[3] = 1;
    for (int mu = 2; mu >= 0; --mu) {
        g.lstr[mu] = g.lstr[mu + 1] * b[mu + 1];
        g.bstr[mu] = g.bstr[mu + 1] * g.nb[mu + 1];
    }
    g.Vb = b[0] * b[1] * b[2] * b[3];
    g.Nb = g.nb[0] * g.nb[1] * g.nb[2] * g.nb[3];
    g.V = (long)g.Vb * g.Nb;
    g.tsign = 1;
    return g;
}

// block coordinates n and in-block coordinates y of a native site
__host__ __device__ inline void site_decompose(const Geom& g, long s, int n[4], int y[4])
{
    int blk = (int)(s / g.Vb);
    int loc = (int)(s - (long)blk * g.Vb);
#pragma unroll
    for (int mu = 3; mu >= 1; --mu) {
        int q = loc / g.b[mu];
        y[mu] = loc - q * g.b[mu];
        loc = q;
        int p = blk / g.nb[mu];
        n[mu] = blk - p * g.nb[mu];
        blk = p;
    }
    y[0] = loc;
    n[0] = blk;
}

__host__ __device__ inline long site_compose(const Geom& g, const int n[4], const int y[4])
{
    long blk = ((long)(n[0] * g.nb[1] + n[1]) * g.nb[2] + n[2]) * g.nb[3] + n[3];
    long loc = ((long)(y[0] * g.b[1] + y[1]) * g.b[2] + y[2]) * g.b[3] + y[3];
    return blk * g.Vb + loc;
}

// The same site in the transposed in-block order (y0 fastest, y3 slowest),
// blocks in the native order: a copy of a field in this order holds the faces
// {y_3 = const} of a 4^4 block as whole 64-site tiles and the faces
// {y_2 = const} as runs of 16 sites, which the native order scatters.
__host__ __device__ inline long site_compose_t(const Geom& g, const int n[4], const int y[4])
{
    long blk = ((long)(n[0] * g.nb[1] + n[1]) * g.nb[2] + n[2]) * g.nb[3] + n[3];
    long loc = ((long)(y[3] * g.b[2] + y[2]) * g.b[1] + y[1]) * g.b[0] + y[0];
    return blk * g.Vb + loc;
}

// native index of the neighbour s + step*mu (step = +1 or -1), periodic
__host__ __device__ inline long site_step(const Geom& g, long s, const int n[4], const int y[4], int mu, int step)
{
    int yy = y[mu] + step;
    if (yy >= 0 && yy < g.b[mu])
        return s + (long)step * g.lstr[mu];
    // leave the block: wrap y, move the block coordinate with periodic wrap
    int nn = n[mu] + step;
    int dn = step;
    if (nn < 0) {
        dn += g.nb[mu];
    } else if (nn >= g.nb[mu]) {
        dn -= g.nb[mu];
    }
    long dy = (step > 0) ? -(long)(g.b[mu] - 1) * g.lstr[mu] : (long)(g.b[mu] - 1) * g.lstr[mu];
    return s + (long)dn * g.bstr[mu] * g.Vb + dy;
}

// whether the hop from a site with block/in-block coordinates (n, y) in
// direction mu, orientation step, crosses the time boundary x0 = L0-1 <-> 0
// (where an antiperiodic quark field picks up a factor -1)
__host__ __device__ inline bool crosses_time(const Geom& g, const int n[4], const int y[4], int mu, int step)
{
    if (mu != 0 || g.tsign > 0)
        return false;
    return step > 0 ? (n[0] == g.nb[0] - 1 && y[0] == g.b[0] - 1) : (n[0] == 0 && y[0] == 0);
}

// canonical site index from global coordinates
__host__ __device__ inline long canon_index(const Geom& g, const int x[4])
{
    return (((long)x[0] * g.L[1] + x[1]) * g.L[2] + x[2]) * g.L[3] + x[3];
}

// --------------------------------------------------- XCD-aware numbering
//
// Workgroups are handed to the 8 XCDs round robin by id. Renumber so that
// XCD k works on the contiguous id range [k*per, (k+1)*per): neighbouring
// sites then share one XCD's L2. The grid must be padded to a multiple of 8;
// ids >= the real count do nothing.
constexpr int kNumXcd = 8;

__device__ inline int xcd_remap(int bid, int grid_padded)
{
    int per = grid_padded / kNumXcd;
    return (bid % kNumXcd) * per + bid / kNumXcd;
}

__host__ inline int pad_grid(long nwg) { return (int)(((nwg + kNumXcd - 1) / kNumXcd) * kNumXcd); }

// --------------------------------------------------------- reductions

// Sum over the 64 lanes of a wavefront, the same value in every lane; every
// lane must be active. Cross-lane moves go through DPP: swaps inside quads,
// the half-row and row mirrors (16-lane sums in every lane), then row 0's and
// row 2's last lanes are broadcast into rows 1 and 3, and lane 31 into rows 2
// and 3, which leaves the total in lane 63; a readlane hands it to all.
namespace wave_detail {
template <int CTRL, int ROWS> __device__ inline int dpp(int v)
{
    // lanes of rows outside ROWS (and lanes without a source) receive 0
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS> __device__ inline double dpp(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp<CTRL, ROWS>((int)b), hi = dpp<CTRL, ROWS>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL, int ROWS> __device__ inline float dpp(float v)
{
    return __int_as_float(dpp<CTRL, ROWS>(__float_as_int(v)));
}
__device__ inline double lane63(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline float lane63(float v) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63)); }
}  // namespace wave_detail

template <typename T> __device__ inline T wave_sum(T v)
{
    using namespace wave_detail;
    v += dpp<0xB1, 0xF>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp<0x4E, 0xF>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp<0x141, 0xF>(v);  // row_half_mirror
    v += dpp<0x140, 0xF>(v);  // row_mirror
    v += dpp<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return lane63(v);
}

// Sum of v over the workgroup (blockDim.x a multiple of 64, <= 1024); every
// thread receives the result. scratch holds >= 16 T. Fixed order: deterministic.
template <typename T> __device__ inline T block_sum(T v, T* scratch)
{
    v = wave_sum(v);
    int lane = threadIdx.x & 63;
    int wid = threadIdx.x >> 6;
    int nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0)
        scratch[wid] = v;
    __syncthreads();
    T r = 0;
    for (int i = 0; i < nw; ++i)
        r += scratch[i];
    return r;
}

}  // namespace dfl
