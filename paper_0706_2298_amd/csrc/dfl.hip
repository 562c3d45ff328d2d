// Block-projection kernels of the deflation subspace (sections 4.1-4.2 and
// appendix A.1). The deflation blocks are the layout blocks, so every block
// is a contiguous run of Vb sites in each of the 12 planes: one workgroup per
// block reads its block of every basis field with unit stride.
#include "internal.h"

namespace dfl {

namespace {

constexpr int kBT = 256;  // threads per block-kernel workgroup

// w[blk*Ns + k] = sum_{x in blk} sum_c conj(Phi_k(x,c)) psi(x,c)   (eq. (4.1))
__global__ __launch_bounds__(kBT) void k_restrict(Geom g, const c64* __restrict__ Phi, int Ns,
                                                  const c64* __restrict__ psi, c64* __restrict__ w)
{
    __shared__ double part[2 * 64][kBT / 64];
    const int blk = blockIdx.x;
    const long base = (long)blk * g.Vb;
    const long fs = 12 * g.V;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int k0 = 0; k0 < Ns; k0 += 64) {
        int kn = Ns - k0 < 64 ? Ns - k0 : 64;
        for (int kk = 0; kk < kn; ++kk) {
            const c64* ph = Phi + (long)(k0 + kk) * fs;
            double re = 0.0, im = 0.0;
            for (int t = threadIdx.x; t < g.Vb; t += kBT) {
                long s = base + t;
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    c64 a = ph[tidx(s, c, 12)];
                    c64 b = psi[tidx(s, c, 12)];
                    re += a.re * b.re + a.im * b.im;
                    im += a.re * b.im - a.im * b.re;
                }
            }
            re = wave_sum(re);
            im = wave_sum(im);
            if (lane == 0) {
                part[2 * kk][wid] = re;
                part[2 * kk + 1][wid] = im;
            }
        }
        __syncthreads();
        if (threadIdx.x < 2 * kn) {
            double t = 0.0;
            for (int q = 0; q < kBT / 64; ++q)
                t += part[threadIdx.x][q];
            double* dst = reinterpret_cast<double*>(w + (long)blk * Ns + k0);
            dst[threadIdx.x] = t;
        }
        __syncthreads();
    }
}

// psi(x) = sum_k Phi_k(x) v[blk*Ns + k]
__global__ __launch_bounds__(256) void k_prolong(Geom g, const c64* __restrict__ Phi, int Ns,
                                                 const c64* __restrict__ v, c64* __restrict__ psi)
{
    long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V)
        return;
    long blk = s / g.Vb;
    const long fs = 12 * g.V;
    c64 acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c)
        acc[c] = c64{0.0, 0.0};
    for (int k = 0; k < Ns; ++k) {
        c64 vk = v[blk * Ns + k];
        const c64* ph = Phi + (long)k * fs;
#pragma unroll
        for (int c = 0; c < 12; ++c)
            acc[c] += ph[tidx(s, c, 12)] * vk;
    }
#pragma unroll
    for (int c = 0; c < 12; ++c)
        psi[tidx(s, c, 12)] = acc[c];
}

// Modified Gram-Schmidt per block, in place, order l = 0..Ns-1 (eq. (4.2)).
// flag is set to 1 if a block loses rank.
__global__ __launch_bounds__(kBT) void k_block_gs(Geom g, c64* __restrict__ F, int Ns, double rank_tol,
                                                  int* __restrict__ flag)
{
    __shared__ double sh[8];
    const long base = (long)blockIdx.x * g.Vb;
    const long fs = 12 * g.V;
    for (int l = 0; l < Ns; ++l) {
        c64* fl = F + (long)l * fs;
        // norm of the restricted input field (for the rank test)
        double n0 = 0.0;
        for (int t = threadIdx.x; t < g.Vb; t += kBT)
            for (int c = 0; c < 12; ++c) {
                c64 a = fl[tidx(base + t, c, 12)];
                n0 += a.re * a.re + a.im * a.im;
            }
        n0 = block_sum(n0, sh);
        for (int k = 0; k < l; ++k) {
            const c64* fk = F + (long)k * fs;
            double re = 0.0, im = 0.0;
            for (int t = threadIdx.x; t < g.Vb; t += kBT)
                for (int c = 0; c < 12; ++c) {
                    long i = tidx(base + t, c, 12);
                    c64 a = fk[i], b = fl[i];
                    re += a.re * b.re + a.im * b.im;
                    im += a.re * b.im - a.im * b.re;
                }
            re = block_sum(re, sh);
            im = block_sum(im, sh);
            c64 cf{re, im};
            for (int t = threadIdx.x; t < g.Vb; t += kBT)
                for (int c = 0; c < 12; ++c) {
                    long i = tidx(base + t, c, 12);
                    fl[i] -= cf * fk[i];
                }
        }
        double nv = 0.0;
        for (int t = threadIdx.x; t < g.Vb; t += kBT)
            for (int c = 0; c < 12; ++c) {
                c64 a = fl[tidx(base + t, c, 12)];
                nv += a.re * a.re + a.im * a.im;
            }
        nv = sqrt(block_sum(nv, sh));
        n0 = sqrt(n0);
        if (!(nv > rank_tol * n0) || !(n0 > 0.0)) {
            if (threadIdx.x == 0)
                atomicOr(flag, 2);
            nv = 1.0;
        }
        double inv = 1.0 / nv;
        for (int t = threadIdx.x; t < g.Vb; t += kBT)
            for (int c = 0; c < 12; ++c) {
                long i = tidx(base + t, c, 12);
                fl[i].re *= inv;
                fl[i].im *= inv;
            }
    }
}

// A[blk][d][k][l] = sum_{x in blk} conj(Phi_k(x)) Y(x) for all k, fixed d, l
__global__ __launch_bounds__(kBT) void k_little_column(Geom g, const c64* __restrict__ Phi, int Ns,
                                                       const c64* __restrict__ Y, c64* __restrict__ A, int d, int l)
{
    __shared__ double part[2][kBT / 64];
    const long base = (long)blockIdx.x * g.Vb;
    const long fs = 12 * g.V;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int k = 0; k < Ns; ++k) {
        const c64* ph = Phi + (long)k * fs;
        double re = 0.0, im = 0.0;
        for (int t = threadIdx.x; t < g.Vb; t += kBT)
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                long i = tidx(base + t, c, 12);
                c64 a = ph[i], b = Y[i];
                re += a.re * b.re + a.im * b.im;
                im += a.re * b.im - a.im * b.re;
            }
        re = wave_sum(re);
        im = wave_sum(im);
        __syncthreads();
        if (lane == 0) {
            part[0][wid] = re;
            part[1][wid] = im;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = 0.0, b = 0.0;
            for (int q = 0; q < kBT / 64; ++q) {
                a += part[0][q];
                b += part[1][q];
            }
            A[(((long)blockIdx.x * 9 + d) * Ns + k) * Ns + l] = c64{a, b};
        }
    }
}

// w[blk] = sum_d A[blk][d] v[nbr_d(blk)], one thread per (blk, k) row
template <typename T>
__global__ __launch_bounds__(256) void k_little_apply(Geom g, const cpx<T>* __restrict__ A, int Ns,
                                                      const cpx<T>* __restrict__ v, cpx<T>* __restrict__ w)
{
    long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= (long)g.Nb * Ns)
        return;
    int blk = (int)(row / Ns);
    int k = (int)(row - (long)blk * Ns);
    int n[4];
    int rest = blk;
    for (int mu = 3; mu >= 0; --mu) {
        n[mu] = rest % g.nb[mu];
        rest /= g.nb[mu];
    }
    double re = 0.0, im = 0.0;
    for (int d = 0; d < 9; ++d) {
        int nbr = blk;
        if (d > 0) {
            int mu = (d - 1) >> 1;
            int step = (d & 1) ? +1 : -1;
            int nn = n[mu] + step;
            if (nn < 0)
                nn += g.nb[mu];
            if (nn >= g.nb[mu])
                nn -= g.nb[mu];
            nbr = blk + (nn - n[mu]) * g.bstr[mu];
        }
        const cpx<T>* a = A + (((long)blk * 9 + d) * Ns + k) * Ns;
        const cpx<T>* x = v + (long)nbr * Ns;
        for (int l = 0; l < Ns; ++l) {
            cpx<T> p = a[l], q = x[l];
            re += (double)p.re * (double)q.re - (double)p.im * (double)q.im;
            im += (double)p.re * (double)q.im + (double)p.im * (double)q.re;
        }
    }
    w[row] = cpx<T>{(T)re, (T)im};
}

__global__ void k_little_shift(Geom g, c64* A, int Ns, double dm)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)g.Nb * Ns)
        return;
    long blk = i / Ns, k = i - blk * Ns;
    A[((blk * 9) * Ns + k) * Ns + k].re += dm;
}

// A32[i] = A[i]; At[blk][d][l][k] = A[blk][d][k][l]
__global__ void k_little_copies(const c64* __restrict__ A, c32* A32, c64* At64, c32* At32, long nblocks, int Ns)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long n = nblocks * Ns * Ns;
    if (i >= n)
        return;
    long bd = i / ((long)Ns * Ns);
    int rem = (int)(i - bd * Ns * Ns);
    int k = rem / Ns, l = rem - k * Ns;
    c64 v = A[i];
    A32[i] = c32{(float)v.re, (float)v.im};
    long j = bd * Ns * Ns + (long)l * Ns + k;
    At64[j] = v;
    At32[j] = c32{(float)v.re, (float)v.im};
}

__global__ void k_c64_to_c32(const c64* a, c32* b, long n)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        b[i] = c32{(float)a[i].re, (float)a[i].im};
}

}  // namespace

void launch_restrict64(const Geom& g, const c64* Phi, int Ns, const c64* psi, c64* w, hipStream_t s)
{
    hipLaunchKernelGGL(k_restrict, dim3(g.Nb), dim3(kBT), 0, s, g, Phi, Ns, psi, w);
}
void launch_prolong64(const Geom& g, const c64* Phi, int Ns, const c64* v, c64* psi, hipStream_t s)
{
    hipLaunchKernelGGL(k_prolong, dim3((unsigned)((g.V + 255) / 256)), dim3(256), 0, s, g, Phi, Ns, v, psi);
}
void launch_block_gs64(const Geom& g, c64* F, int Ns, double rank_tol, int* flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_block_gs, dim3(g.Nb), dim3(kBT), 0, s, g, F, Ns, rank_tol, flag);
}
void launch_little_column64(const Geom& g, const c64* Phi, int Ns, const c64* Y, c64* A, int d, int l, hipStream_t s)
{
    hipLaunchKernelGGL(k_little_column, dim3(g.Nb), dim3(kBT), 0, s, g, Phi, Ns, Y, A, d, l);
}
template <typename T>
void launch_little_apply(const Geom& g, const cpx<T>* A, int Ns, const cpx<T>* v, cpx<T>* w, hipStream_t s)
{
    long rows = (long)g.Nb * Ns;
    hipLaunchKernelGGL(k_little_apply<T>, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, g, A, Ns, v, w);
}
template void launch_little_apply<double>(const Geom&, const c64*, int, const c64*, c64*, hipStream_t);
template void launch_little_apply<float>(const Geom&, const c32*, int, const c32*, c32*, hipStream_t);

void launch_little_shift(const Geom& g, c64* A, int Ns, double dm, hipStream_t s)
{
    long n = (long)g.Nb * Ns;
    hipLaunchKernelGGL(k_little_shift, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, A, Ns, dm);
}
void launch_little_copies(const c64* A, c32* A32, c64* At64, c32* At32, long nblocks, int Ns, hipStream_t s)
{
    long n = nblocks * Ns * Ns;
    if (n > 0)
        hipLaunchKernelGGL(k_little_copies, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, A32, At64, At32,
                           nblocks, Ns);
}
void launch_c64_to_c32(const c64* a, c32* b, long n, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_c64_to_c32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n);
}

}  // namespace dfl
