// Canonical <-> native conversions of quark fields, and link compression.
//
// Canonical quark field: complex128 [V][12] in lexicographic site order.
// Native quark field: 64-site tiles of 12 components in block-major site
// order (common.h). Links: FP64, FP32 and BF16 store the first two rows only
// (24 entries per site), the third row being rebuilt as conj(row0 x row1),
// which is exact for SU(3) matrices.
#include <algorithm>

#include "internal.h"

namespace dfl {

namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_pack_field(Geom g, const c64* __restrict__ canon,
                                                    cpx<T>* __restrict__ nat, int nrhs)
{
    long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    int r = blockIdx.y;
    if (s >= g.V || r >= nrhs)
        return;
    int n[4], y[4], x[4];
    site_decompose(g, s, n, y);
    for (int mu = 0; mu < 4; ++mu)
        x[mu] = n[mu] * g.b[mu] + y[mu];
    long c = canon_index(g, x);
    const c64* src = canon + ((long)r * g.V + c) * 12;
    cpx<T>* dst = nat + (long)r * 12 * g.V;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        c64 v = src[k];
        dst[tidx(s, k, 12)] = cpx<T>{(T)v.re, (T)v.im};
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_unpack_field(Geom g, const cpx<T>* __restrict__ nat,
                                                      c64* __restrict__ canon, int nrhs)
{
    long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    int r = blockIdx.y;
    if (s >= g.V || r >= nrhs)
        return;
    int n[4], y[4], x[4];
    site_decompose(g, s, n, y);
    for (int mu = 0; mu < 4; ++mu)
        x[mu] = n[mu] * g.b[mu] + y[mu];
    long c = canon_index(g, x);
    c64* dst = canon + ((long)r * g.V + c) * 12;
    const cpx<T>* src = nat + (long)r * 12 * g.V;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        cpx<T> v = src[tidx(s, k, 12)];
        dst[k] = c64{(double)v.re, (double)v.im};
    }
}

// round-to-nearest-even float -> bfloat16 bits (finite inputs)
__device__ inline uint32_t bf16_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return u >> 16;
}

// Links in two-row form ([4][6] entries per site) in FP64, FP32 and BF16; the
// third row is rebuilt as conj(row0 x row1) wherever a link is used. flag |= 1
// where the given third row differs from that (the link is not SU(3)).
__global__ __launch_bounds__(256) void k_pack_gauge(Geom g, const c64* __restrict__ canon, c64* U64, c32* U32,
                                                    uint32_t* Ubf, int* flag)
{
    long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V)
        return;
    int n[4], y[4], x[4];
    site_decompose(g, s, n, y);
    for (int mu = 0; mu < 4; ++mu)
        x[mu] = n[mu] * g.b[mu] + y[mu];
    long c = canon_index(g, x);
    bool bad = false;
    for (int mu = 0; mu < 4; ++mu) {
        const c64* src = canon + (c * 4 + mu) * 9;
        c64 u[9];
        for (int k = 0; k < 9; ++k)
            u[k] = src[k];
        double scale = 0.0;
        for (int k = 0; k < 6; ++k) {
            const c64 v = u[k];
            scale += v.re * v.re + v.im * v.im;
            if (U64)
                U64[tidx(s, mu * 6 + k, 24)] = v;
            if (U32)
                U32[tidx(s, mu * 6 + k, 24)] = c32{(float)v.re, (float)v.im};
            if (Ubf)
                Ubf[tidx(s, mu * 6 + k, 24)] = bf16_bits((float)v.re) | (bf16_bits((float)v.im) << 16);
        }
        for (int b = 0; b < 3; ++b) {
            const int b1 = (b + 1) % 3, b2 = (b + 2) % 3;
            const c64 r = conjg(u[b1] * u[3 + b2] - u[b2] * u[3 + b1]);
            const double dr = r.re - u[6 + b].re, di = r.im - u[6 + b].im;
            bad |= !(dr * dr + di * di <= 1e-24 * (1.0 + scale * scale));
        }
    }
    if (bad)
        atomicOr(flag, 1);
}

__global__ __launch_bounds__(256) void k_f64_to_f32(const c64* __restrict__ in, c32* __restrict__ out, long n)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = c32{(float)in[i].re, (float)in[i].im};
}

// out_b = in_b / sqrt(nrm2[b * cstride]) rounded to FP32 (the product in FP64),
// field b of n entries at b * n; blockIdx.y = field. With flag non-null, bit 1
// of *flag is set if an input entry is not finite.
__global__ __launch_bounds__(256) void k_to_f32_scaled(const c64* __restrict__ in, c32* __restrict__ out, long n,
                                                       const double* __restrict__ nrm2, int cstride, int* flag)
{
    const int b = blockIdx.y;
    const double q = nrm2[(long)b * cstride];
    const double f = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
    in += (long)b * n;
    out += (long)b * n;
    bool bad = false;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const c64 z = in[i];
        bad |= !isfinite(z.re) || !isfinite(z.im);
        out[i] = c32{(float)(z.re * f), (float)(z.im * f)};
    }
    if (flag && bad)
        atomicOr(flag, 1);
}

__global__ __launch_bounds__(256) void k_f32_to_f64(const c32* __restrict__ in, c64* __restrict__ out, long n)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = c64{(double)in[i].re, (double)in[i].im};
}

inline dim3 site_grid(const Geom& g, int nrhs) { return dim3((unsigned)((g.V + 255) / 256), (unsigned)nrhs); }

}  // namespace

void launch_pack_field64(const Geom& g, const c64* canon, c64* nat, int nrhs, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_field<double>, site_grid(g, nrhs), dim3(256), 0, s, g, canon, nat, nrhs);
}
void launch_pack_field32(const Geom& g, const c64* canon, c32* nat, int nrhs, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_field<float>, site_grid(g, nrhs), dim3(256), 0, s, g, canon, nat, nrhs);
}
void launch_unpack_field64(const Geom& g, const c64* nat, c64* canon, int nrhs, hipStream_t s)
{
    hipLaunchKernelGGL(k_unpack_field<double>, site_grid(g, nrhs), dim3(256), 0, s, g, nat, canon, nrhs);
}
void launch_unpack_field32(const Geom& g, const c32* nat, c64* canon, int nrhs, hipStream_t s)
{
    hipLaunchKernelGGL(k_unpack_field<float>, site_grid(g, nrhs), dim3(256), 0, s, g, nat, canon, nrhs);
}
void launch_pack_gauge(const Geom& g, const c64* canon, c64* U64, c32* U32, uint32_t* Ubf, int* flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_gauge, site_grid(g, 1), dim3(256), 0, s, g, canon, U64, U32, Ubf, flag);
}
void launch_f64_to_f32(const c64* in, c32* out, long n, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_f64_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, n);
}
void launch_f64_to_f32_scaled(const c64* in, c32* out, long n, int nb, const double* nrm2, int cstride, hipStream_t s,
                              int* finite_flag)
{
    if (n > 0 && nb > 0) {
        const long blocks = std::min<long>((n + 255) / 256, 4096);
        hipLaunchKernelGGL(k_to_f32_scaled, dim3((unsigned)blocks, (unsigned)nb), dim3(256), 0, s, in, out, n,
                           nrm2, cstride, finite_flag);
    }
}
void launch_f32_to_f64(const c32* in, c64* out, long n, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_f32_to_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, n);
}

}  // namespace dfl
