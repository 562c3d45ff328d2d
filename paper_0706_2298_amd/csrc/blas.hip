// Vector kernels of the Krylov solvers: copies, fused multi-dot products,
// multi-axpy with coefficients read from device memory, norms.
//
// Reductions are two-pass with a fixed grid (kRedBlocks workgroups, grid-
// stride loops) and a fixed summation tree, accumulated in FP64, so results
// are bit-reproducible run to run and independent of stream timing.
#include "internal.h"

namespace dfl {

namespace {

constexpr int kChunk = 8;  // vectors per pass of the multi-dot

template <typename T> __global__ __launch_bounds__(256) void k_zero(cpx<T>* x, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        x[i] = cpx<T>{0, 0};
}

template <typename T> __global__ __launch_bounds__(256) void k_copy(const cpx<T>* __restrict__ x, cpx<T>* __restrict__ y, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        y[i] = x[i];
}

template <typename T>
__global__ __launch_bounds__(256) void k_sub(const cpx<T>* __restrict__ x, const cpx<T>* __restrict__ y,
                                             cpx<T>* __restrict__ z, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        z[i] = cpx<T>{x[i].re - y[i].re, x[i].im - y[i].im};
}

template <typename T>
__global__ __launch_bounds__(256) void k_add(const cpx<T>* __restrict__ x, const cpx<T>* __restrict__ y,
                                             cpx<T>* __restrict__ z, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        z[i] = cpx<T>{x[i].re + y[i].re, x[i].im + y[i].im};
}

// Batched forms: blockIdx.y is the right-hand side b; vectors of RHS b sit
// at a fixed offset (xb, yb) from those of RHS 0, its partial sums at
// b * kMaxDot * kRedBlocks * 2, its results at dst + b * dstride. A non-null
// mask skips every RHS b with active[b] == 0 (nothing is read or written).

// partial[(b*kMaxDot + j0 + j)*kRedBlocks + blockIdx)*2 + {0,1}] = this workgroup's share of (X_j, y)
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_multidot_partial(const cpx<T>* __restrict__ X, long stride, int j0,
                                                                  int m, const cpx<T>* __restrict__ y, long n,
                                                                  long xb, long yb, const int* __restrict__ active,
                                                                  double* __restrict__ partial)
{
    const int b = blockIdx.y;
    if (active && !active[b])
        return;
    X += b * xb;
    y += b * yb;
    partial += (long)b * kMaxDot * kRedBlocks * 2;
    __shared__ double sh[2 * kChunk][kRedThreads / 64];
    double re[kChunk], im[kChunk];
#pragma unroll
    for (int j = 0; j < kChunk; ++j)
        re[j] = im[j] = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        cpx<T> bv = y[i];
        double br = (double)bv.re, bi = (double)bv.im;
#pragma unroll
        for (int j = 0; j < kChunk; ++j) {
            if (j < m) {
                cpx<T> a = X[(long)(j0 + j) * stride + i];
                double ar = (double)a.re, ai = (double)a.im;
                re[j] += ar * br + ai * bi;
                im[j] += ar * bi - ai * br;
            }
        }
    }
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < kChunk; ++j) {
        double a = wave_sum(re[j]);
        double c = wave_sum(im[j]);
        if (lane == 0) {
            sh[2 * j][wid] = a;
            sh[2 * j + 1][wid] = c;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * m) {
        double t = 0.0;
        for (int w = 0; w < kRedThreads / 64; ++w)
            t += sh[threadIdx.x][w];
        int j = threadIdx.x >> 1, c = threadIdx.x & 1;
        partial[((long)(j0 + j) * kRedBlocks + blockIdx.x) * 2 + c] = t;
    }
}

// dst[b*dstride + jc] = sum over workgroups of RHS b's partials, jc < 2m
// (jc = 2j + {0: re, 1: im}); one wavefront per value, a fixed lane-strided
// order and wavefront tree. Grid: (ceil(2m / 4), nrhs) workgroups of 256.
__global__ __launch_bounds__(256) void k_reduce_partials(const double* __restrict__ partial, int m,
                                                         double* __restrict__ dst, int dstride,
                                                         const int* __restrict__ active)
{
    const int b = blockIdx.y;
    if (active && !active[b])
        return;
    const int lane = threadIdx.x & 63;
    const int jc = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (jc >= 2 * m)
        return;  // whole wavefronts
    partial += (long)b * kMaxDot * kRedBlocks * 2;
    const int j = jc >> 1, c = jc & 1;
    double t = 0.0;
    for (int q = lane; q < kRedBlocks; q += 64)
        t += partial[((long)j * kRedBlocks + q) * 2 + c];
    t = wave_sum(t);
    if (lane == 0)
        dst[(long)b * dstride + jc] = t;
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_norm2_partial(const cpx<T>* __restrict__ x, long n, long xb,
                                                               const int* __restrict__ active,
                                                               double* __restrict__ partial)
{
    const int b = blockIdx.y;
    if (active && !active[b])
        return;
    x += b * xb;
    partial += (long)b * kMaxDot * kRedBlocks * 2;
    __shared__ double sh[4];
    double t = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        double a = (double)x[i].re, c = (double)x[i].im;
        t += a * a + c * c;
    }
    t = block_sum(t, sh);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = t;
        partial[2 * blockIdx.x + 1] = 0.0;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_multiaxpy(const cpx<T>* __restrict__ X, long stride, int m,
                                                   const double* __restrict__ coef, int cstride, double sign,
                                                   cpx<T>* __restrict__ y, long n, long xb, long yb,
                                                   const int* __restrict__ active)
{
    const int b = blockIdx.y;
    if (active && !active[b])
        return;
    X += b * xb;
    y += b * yb;
    coef += (long)b * cstride;
    __shared__ double c[2 * kMaxDot];
    for (int j = threadIdx.x; j < 2 * m; j += blockDim.x)
        c[j] = sign * coef[j];
    __syncthreads();
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        double yr = (double)y[i].re, yi = (double)y[i].im;
        for (int j = 0; j < m; ++j) {
            cpx<T> a = X[(long)j * stride + i];
            double ar = (double)a.re, ai = (double)a.im;
            yr += c[2 * j] * ar - c[2 * j + 1] * ai;
            yi += c[2 * j] * ai + c[2 * j + 1] * ar;
        }
        y[i] = cpx<T>{(T)yr, (T)yi};
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_scale_invsqrt(cpx<T>* __restrict__ x, long n, long xb,
                                                       const double* __restrict__ nrm2, int cstride,
                                                       const int* __restrict__ active)
{
    const int b = blockIdx.y;
    if (active && !active[b])
        return;
    x += b * xb;
    const double q = nrm2[(long)b * cstride];
    const double f = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        x[i].re = (T)((double)x[i].re * f);
        x[i].im = (T)((double)x[i].im * f);
    }
}

// The closing steps of a GCR step on source b (vectors at offset b * xb):
// partials of ||x||^2 (slot 0, imaginary part 0) and of (x, y) (slot 1) in
// one pass over x and y.
__global__ __launch_bounds__(kRedThreads) void k_norm_dot_partial(const c64* __restrict__ x, const c64* __restrict__ y,
                                                                  long n, long xb, const int* __restrict__ active,
                                                                  double* __restrict__ partial)
{
    const int b = blockIdx.y;
    if (active && !active[b])
        return;
    x += b * xb;
    y += b * xb;
    partial += (long)b * kMaxDot * kRedBlocks * 2;
    __shared__ double sh[16];
    double nn = 0.0, dr = 0.0, di = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const c64 a = x[i], c = y[i];
        nn += a.re * a.re + a.im * a.im;
        dr += a.re * c.re + a.im * c.im;
        di += a.re * c.im - a.im * c.re;
    }
    nn = block_sum(nn, sh);
    dr = block_sum(dr, sh);
    di = block_sum(di, sh);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = nn;
        partial[2 * blockIdx.x + 1] = 0.0;
        partial[(kRedBlocks + blockIdx.x) * 2] = dr;
        partial[(kRedBlocks + blockIdx.x) * 2 + 1] = di;
    }
}

// With sc = {||x||^2, 0, Re (x, y), Im (x, y)} of source b (at b * cstride):
// y <- y - ((x, y) / ||x||^2) x, x <- x / ||x||, and partials of the new
// ||y||^2 (slot 0), in one pass.
__global__ __launch_bounds__(kRedThreads) void k_scale_update_partial(c64* __restrict__ x, c64* __restrict__ y, long n,
                                                                      long xb, const double* __restrict__ sc,
                                                                      int cstride, const int* __restrict__ active,
                                                                      double* __restrict__ partial)
{
    const int b = blockIdx.y;
    if (active && !active[b])
        return;
    x += b * xb;
    y += b * xb;
    sc += (long)b * cstride;
    partial += (long)b * kMaxDot * kRedBlocks * 2;
    __shared__ double sh[16];
    const double q = sc[0];
    const double f = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
    const double cr = q > 0.0 ? sc[2] / q : 0.0, ci = q > 0.0 ? sc[3] / q : 0.0;
    double t = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const c64 a = x[i], c = y[i];
        const double yr = c.re - (cr * a.re - ci * a.im);
        const double yi = c.im - (cr * a.im + ci * a.re);
        y[i] = c64{yr, yi};
        x[i] = c64{a.re * f, a.im * f};
        t += yr * yr + yi * yi;
    }
    t = block_sum(t, sh);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = t;
        partial[2 * blockIdx.x + 1] = 0.0;
    }
}

__global__ void k_add_scalars(const double* a, const double* b, double* dst, int m)
{
    for (int i = threadIdx.x; i < 2 * m; i += blockDim.x)
        dst[i] = a[i] + b[i];
}

template <typename T> __global__ __launch_bounds__(256) void k_finite(const cpx<T>* __restrict__ x, long n, int* flag)
{
    bool bad = false;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        double a = (double)x[i].re, b = (double)x[i].im;
        bad |= !isfinite(a) || !isfinite(b);
    }
    if (bad)
        atomicOr(flag, 1);
}

inline unsigned stream_grid(long n)
{
    long g = (n + 255) / 256;
    if (g > 2048)
        g = 2048;
    if (g < 1)
        g = 1;
    return (unsigned)g;
}

}  // namespace

template <typename T> void launch_zero(cpx<T>* x, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero<T>, dim3(stream_grid(n)), dim3(256), 0, s, x, n);
}
template <typename T> void launch_copy(const cpx<T>* x, cpx<T>* y, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy<T>, dim3(stream_grid(n)), dim3(256), 0, s, x, y, n);
}
template <typename T> void launch_sub(const cpx<T>* x, const cpx<T>* y, cpx<T>* z, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_sub<T>, dim3(stream_grid(n)), dim3(256), 0, s, x, y, z, n);
}

template <typename T> void launch_add(const cpx<T>* x, const cpx<T>* y, cpx<T>* z, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_add<T>, dim3(stream_grid(n)), dim3(256), 0, s, x, y, z, n);
}

template <typename T>
void launch_multidot_b(const cpx<T>* X, long stride, int m, const cpx<T>* y, long n, int nb, long xb, long yb,
                       double* red, double* dst, int dstride, const int* active, hipStream_t s)
{
    if (m <= 0 || nb <= 0)
        return;
    for (int j0 = 0; j0 < m; j0 += kChunk) {
        int mm = m - j0 < kChunk ? m - j0 : kChunk;
        hipLaunchKernelGGL(k_multidot_partial<T>, dim3(kRedBlocks, nb), dim3(kRedThreads), 0, s, X, stride, j0, mm,
                           y, n, xb, yb, active, red);
    }
    hipLaunchKernelGGL(k_reduce_partials, dim3((2 * m + 3) / 4, nb), dim3(256), 0, s, red, m, dst, dstride, active);
}

template <typename T>
void launch_norm2_b(const cpx<T>* x, long n, int nb, long xb, double* red, double* dst, int dstride,
                    const int* active, hipStream_t s)
{
    if (nb <= 0)
        return;
    hipLaunchKernelGGL(k_norm2_partial<T>, dim3(kRedBlocks, nb), dim3(kRedThreads), 0, s, x, n, xb, active, red);
    hipLaunchKernelGGL(k_reduce_partials, dim3(1, nb), dim3(256), 0, s, red, 1, dst, dstride, active);
}

template <typename T>
void launch_multiaxpy_b(const cpx<T>* X, long stride, int m, const double* coef, int cstride, double sign, cpx<T>* y,
                        long n, int nb, long xb, long yb, const int* active, hipStream_t s)
{
    if (m <= 0 || nb <= 0)
        return;
    hipLaunchKernelGGL(k_multiaxpy<T>, dim3(stream_grid(n), nb), dim3(256), 0, s, X, stride, m, coef, cstride, sign,
                       y, n, xb, yb, active);
}

void launch_norm_dot_b(const c64* x, const c64* y, long n, int nb, long xb, double* red, double* dst, int dstride,
                       const int* active, hipStream_t s)
{
    if (nb <= 0)
        return;
    hipLaunchKernelGGL(k_norm_dot_partial, dim3(kRedBlocks, nb), dim3(kRedThreads), 0, s, x, y, n, xb, active, red);
    hipLaunchKernelGGL(k_reduce_partials, dim3(1, nb), dim3(256), 0, s, red, 2, dst, dstride, active);
}

void launch_scale_update_b(c64* x, c64* y, long n, int nb, long xb, const double* sc, int cstride, double* red,
                           double* dst, int dstride, const int* active, hipStream_t s)
{
    if (nb <= 0)
        return;
    hipLaunchKernelGGL(k_scale_update_partial, dim3(kRedBlocks, nb), dim3(kRedThreads), 0, s, x, y, n, xb, sc, cstride,
                       active, red);
    hipLaunchKernelGGL(k_reduce_partials, dim3(1, nb), dim3(256), 0, s, red, 1, dst, dstride, active);
}

template <typename T>
void launch_scale_invsqrt_b(cpx<T>* x, long n, int nb, long xb, const double* nrm2, int cstride, const int* active,
                            hipStream_t s)
{
    if (nb <= 0)
        return;
    hipLaunchKernelGGL(k_scale_invsqrt<T>, dim3(stream_grid(n), nb), dim3(256), 0, s, x, n, xb, nrm2, cstride,
                       active);
}

template <typename T>
void launch_multidot(const cpx<T>* X, long stride, int m, const cpx<T>* y, long n, double* red, double* dst,
                     hipStream_t s)
{
    launch_multidot_b<T>(X, stride, m, y, n, 1, 0, 0, red, dst, 0, nullptr, s);
}

template <typename T> void launch_norm2(const cpx<T>* x, long n, double* red, double* dst, hipStream_t s)
{
    launch_norm2_b<T>(x, n, 1, 0, red, dst, 0, nullptr, s);
}

template <typename T>
void launch_multiaxpy(const cpx<T>* X, long stride, int m, const double* coef, double sign, cpx<T>* y, long n,
                      hipStream_t s)
{
    launch_multiaxpy_b<T>(X, stride, m, coef, 0, sign, y, n, 1, 0, 0, nullptr, s);
}

template <typename T> void launch_scale_invsqrt(cpx<T>* x, long n, const double* nrm2, hipStream_t s)
{
    launch_scale_invsqrt_b<T>(x, n, 1, 0, nrm2, 0, nullptr, s);
}

namespace {
// Gram-Schmidt re-orthogonalisation test per source b: the first pass left
// (x_j, y) for j < k and (y, y) at a1[b*stride + 2j] (j <= k). A second pass
// is needed only if the first cancelled more than 99% of ||y||^2; sources that
// skip it get zero second-pass coefficients (a2) and act2[b] = 0.
__global__ void k_second_pass_mask(const double* __restrict__ a1, double* __restrict__ a2, int k, int stride,
                                   const int* __restrict__ active, int nb, int* __restrict__ act2)
{
    const int b = threadIdx.x;
    if (b >= nb)
        return;
    const double* p = a1 + (long)b * stride;
    double q = 0.0;
    for (int j = 0; j < k; ++j)
        q += p[2 * j] * p[2 * j] + p[2 * j + 1] * p[2 * j + 1];
    const double n2 = p[2 * k];
    const int need = (!active || active[b]) && !(n2 - q >= 0.01 * n2);
    act2[b] = need;
    if (!need)
        for (int j = 0; j < 2 * k; ++j)
            a2[(long)b * stride + j] = 0.0;
}
}  // namespace

void launch_second_pass_mask(const double* a1, double* a2, int k, int stride, const int* active, int nb, int* act2,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_second_pass_mask, dim3(1), dim3(64), 0, s, a1, a2, k, stride, active, nb, act2);
}

void launch_add_scalars(const double* a, const double* b, double* dst, int m, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_scalars, dim3(1), dim3(128), 0, s, a, b, dst, m);
}

template <typename T> void launch_finite_check(const cpx<T>* x, long n, int* flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_finite<T>, dim3(stream_grid(n)), dim3(256), 0, s, x, n, flag);
}

#define INST(T)                                                                                                    \
    template void launch_zero<T>(cpx<T>*, long, hipStream_t);                                                     \
    template void launch_copy<T>(const cpx<T>*, cpx<T>*, long, hipStream_t);                                      \
    template void launch_sub<T>(const cpx<T>*, const cpx<T>*, cpx<T>*, long, hipStream_t);                        \
    template void launch_add<T>(const cpx<T>*, const cpx<T>*, cpx<T>*, long, hipStream_t);                        \
    template void launch_multidot<T>(const cpx<T>*, long, int, const cpx<T>*, long, double*, double*, hipStream_t); \
    template void launch_norm2<T>(const cpx<T>*, long, double*, double*, hipStream_t);                            \
    template void launch_multiaxpy<T>(const cpx<T>*, long, int, const double*, double, cpx<T>*, long, hipStream_t); \
    template void launch_scale_invsqrt<T>(cpx<T>*, long, const double*, hipStream_t);                            \
    template void launch_finite_check<T>(const cpx<T>*, long, int*, hipStream_t);                                 \
    template void launch_multidot_b<T>(const cpx<T>*, long, int, const cpx<T>*, long, int, long, long, double*,    \
                                       double*, int, const int*, hipStream_t);                                    \
    template void launch_norm2_b<T>(const cpx<T>*, long, int, long, double*, double*, int, const int*, hipStream_t); \
    template void launch_multiaxpy_b<T>(const cpx<T>*, long, int, const double*, int, double, cpx<T>*, long, int,  \
                                        long, long, const int*, hipStream_t);                                     \
    template void launch_scale_invsqrt_b<T>(cpx<T>*, long, int, long, const double*, int, const int*, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace dfl
