// GCR for the little system A v = w (eq. (6.1), appendix A.4) in a single
// cooperative launch.
//
// The little vector has Nb*Ns entries; workgroup g owns the blocks
// g, g + G, g + 2G, ... (G = grid size) and all entries of those blocks. One
// GCR step needs three grid-wide barriers:
//   S1  r is complete: reduce ||r||^2, test convergence, then apply
//       chi_k = A r (rows of the owned blocks; the nine neighbour blocks'
//       entries of r are read from global memory);
//   S2  after the first classical Gram-Schmidt pass: reduce (chi_j, chi_k);
//   S3  after the second pass: reduce (chi_j, chi_k'), ||chi_k'||^2,
//       (chi_k', r) and (chi_j, r); the normalised chi_k, its coefficient c_k
//       and the new residue follow without another reduction.
// Partial sums are written per workgroup and every workgroup reduces them in
// the same fixed order, so all workgroups take identical decisions and the
// result is bit-reproducible. After nkv steps (or convergence) the solution
// is updated from the triangular system and the residue recomputed as
// w - A x (two more barriers).
#include <hip/hip_cooperative_groups.h>

#include "internal.h"

namespace cg = cooperative_groups;

namespace dfl {

namespace {

constexpr int LT = 256;
constexpr int NK = kMaxLittleNkv;
// partial-sum slots
constexpr int SA = 0;                 // (chi_j, chi_k), j < k
constexpr int SB = NK;                // (chi_j, chi_k') j<k | (chi_j, r) j<k | ||chi_k'||^2 | (chi_k', r)
constexpr int SC = NK + 2 * NK + 2;   // ||r||^2 inside a cycle
constexpr int SR = SC + 1;            // ||r||^2 after a restart
constexpr int SW = SC + 2;            // ||w||^2
constexpr int NSLOT = SC + 3;

template <typename T> struct LittleArgs {
    Geom g;
    int Ns, nkv, maxiter;
    double tol2;           // stop at ||r||^2 <= tol2 * ||w||^2
    const cpx<T>* At;      // [Nb][9][Ns(l)][Ns(k)]: transposed blocks
    const cpx<T>* w;
    cpx<T>* x;
    cpx<T>* r;
    cpx<T>* xi;            // nkv * N
    cpx<T>* chi;           // nkv * N
    double* part;          // NSLOT * G complex partial sums
    int* stats;            // [0] += iterations, [1] += solves, [2] |= 1 on non-convergence
};

__device__ inline double2 cfma_conj(double2 acc, double ar, double ai, double br, double bi)
{
    // acc += conj(a) * b
    acc.x += ar * br + ai * bi;
    acc.y += ar * bi - ai * br;
    return acc;
}

template <typename T> struct LittleCtx {
    const LittleArgs<T>& a;
    int G, g, t, nbg, R;
    long N;
    __device__ long entry(int e) const
    {
        int i = e / a.Ns;
        int k = e - i * a.Ns;
        return (long)(g + i * G) * a.Ns + k;
    }
};

// reduce slots [s0, s0 + ns) over the G workgroups into red (complex), identically everywhere
__device__ inline void reduce_slots(const double* __restrict__ part, int G, int s0, int ns, double* red)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int s = w; s < ns; s += LT / 64) {
        double re = 0.0, im = 0.0;
        for (int q = lane; q < G; q += 64) {
            re += part[((long)(s0 + s) * G + q) * 2];
            im += part[((long)(s0 + s) * G + q) * 2 + 1];
        }
        re = wave_sum(re);
        im = wave_sum(im);
        if (lane == 0) {
            red[2 * s] = re;
            red[2 * s + 1] = im;
        }
    }
    __syncthreads();
}

// y = A v on the rows this workgroup owns
template <typename T>
__device__ inline void apply_rows(const LittleCtx<T>& c, const cpx<T>* __restrict__ v, cpx<T>* __restrict__ y)
{
    const Geom& g = c.a.g;
    const int Ns = c.a.Ns;
    for (int e = c.t; e < c.R; e += LT) {
        const int i = e / Ns;
        const int k = e - i * Ns;
        const int blk = c.g + i * c.G;
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
                const int mu = (d - 1) >> 1;
                int nn = n[mu] + ((d & 1) ? 1 : -1);
                if (nn < 0)
                    nn += g.nb[mu];
                if (nn >= g.nb[mu])
                    nn -= g.nb[mu];
                nbr = blk + (nn - n[mu]) * g.bstr[mu];
            }
            const cpx<T>* At = c.a.At + ((long)blk * 9 + d) * Ns * Ns + k;
            const cpx<T>* vv = v + (long)nbr * Ns;
            for (int l = 0; l < Ns; ++l) {
                cpx<T> p = At[(long)l * Ns];
                cpx<T> q = vv[l];
                re += (double)p.re * (double)q.re - (double)p.im * (double)q.im;
                im += (double)p.re * (double)q.im + (double)p.im * (double)q.re;
            }
        }
        y[(long)blk * Ns + k] = cpx<T>{(T)re, (T)im};
    }
}

// ||v||^2 over the owned entries -> part[slot][g] (workgroup reduction)
template <typename T>
__device__ inline void partial_norm2(const LittleCtx<T>& c, const cpx<T>* __restrict__ v, int slot, double* sh)
{
    double s = 0.0;
    for (int e = c.t; e < c.R; e += LT) {
        cpx<T> z = v[c.entry(e)];
        s += (double)z.re * (double)z.re + (double)z.im * (double)z.im;
    }
    s = block_sum(s, sh);
    if (c.t == 0) {
        c.a.part[((long)slot * c.G + c.g) * 2] = s;
        c.a.part[((long)slot * c.G + c.g) * 2 + 1] = 0.0;
    }
}

// (X_j, y) for j < m over the owned entries, one thread per j -> part[slot0 + j][g]
template <typename T>
__device__ inline void partial_dots(const LittleCtx<T>& c, const cpx<T>* X, int m, const cpx<T>* __restrict__ y,
                                    int slot0)
{
    if (c.t < m) {
        const cpx<T>* xj = X + (long)c.t * c.N;
        double2 acc = make_double2(0.0, 0.0);
        for (int e = 0; e < c.R; ++e) {
            long i = c.entry(e);
            cpx<T> a = xj[i], b = y[i];
            acc = cfma_conj(acc, (double)a.re, (double)a.im, (double)b.re, (double)b.im);
        }
        c.a.part[((long)(slot0 + c.t) * c.G + c.g) * 2] = acc.x;
        c.a.part[((long)(slot0 + c.t) * c.G + c.g) * 2 + 1] = acc.y;
    }
}

template <typename T> __global__ __launch_bounds__(LT) void k_little_gcr(LittleArgs<T> a)
{
    cg::grid_group grid = cg::this_grid();
    __shared__ double red[2 * (2 * NK + 2)];
    __shared__ double acoef[NK][NK][2];
    __shared__ double bcoef[NK];
    __shared__ double ccoef[NK][2];
    __shared__ double alpha[NK][2];
    __shared__ double sh[8];
    __shared__ double wn2_s, rn2_s;

    LittleCtx<T> c{a, (int)gridDim.x, (int)blockIdx.x, (int)threadIdx.x, 0, 0, (long)a.g.Nb * a.Ns};
    c.nbg = (a.g.Nb - c.g + c.G - 1) / c.G;
    c.R = c.nbg * a.Ns;
    const long N = c.N;

    // x = 0, r = w, ||w||^2
    for (int e = c.t; e < c.R; e += LT) {
        long i = c.entry(e);
        a.x[i] = cpx<T>{0, 0};
        a.r[i] = a.w[i];
    }
    partial_norm2(c, a.w, SW, sh);
    grid.sync();
    reduce_slots(a.part, c.G, SW, 1, red);
    if (c.t == 0)
        wn2_s = red[0];
    __syncthreads();
    const double wn2 = wn2_s;
    int iters = 0;
    bool converged = !(wn2 > 0.0);
    bool broke = false;

    // Every branch below depends only on values reduced identically by all
    // workgroups, so all of them pass the same sequence of grid barriers.
    while (!converged && !broke && iters < a.maxiter) {
        int k = 0;
        for (; k < a.nkv && iters < a.maxiter; ++k) {
            cpx<T>* xk = a.xi + (long)k * N;
            cpx<T>* ck = a.chi + (long)k * N;
            // xi_k = r on the owned entries, and the partial ||r||^2
            for (int e = c.t; e < c.R; e += LT) {
                long i = c.entry(e);
                xk[i] = a.r[i];
            }
            partial_norm2(c, a.r, SC, sh);
            grid.sync();  // S1: r complete everywhere
            reduce_slots(a.part, c.G, SC, 1, red);
            if (c.t == 0)
                rn2_s = red[0];
            __syncthreads();
            if (k > 0 && rn2_s <= a.tol2 * wn2)
                break;  // converged with k directions
            apply_rows(c, xk, ck);
            __syncthreads();
            if (k > 0)
                partial_dots(c, a.chi, k, ck, SA);
            grid.sync();  // S2
            if (k > 0) {
                reduce_slots(a.part, c.G, SA, k, red);
                for (int e = c.t; e < c.R; e += LT) {
                    long i = c.entry(e);
                    double yr = (double)ck[i].re, yi = (double)ck[i].im;
                    for (int j = 0; j < k; ++j) {
                        cpx<T> z = a.chi[(long)j * N + i];
                        yr -= red[2 * j] * (double)z.re - red[2 * j + 1] * (double)z.im;
                        yi -= red[2 * j] * (double)z.im + red[2 * j + 1] * (double)z.re;
                    }
                    ck[i] = cpx<T>{(T)yr, (T)yi};
                }
                if (c.t < k) {
                    acoef[c.t][k][0] = red[2 * c.t];
                    acoef[c.t][k][1] = red[2 * c.t + 1];
                }
                __syncthreads();
            }
            // second pass and the remaining scalars in one reduction
            partial_dots(c, a.chi, k, ck, SB);
            partial_dots(c, a.chi, k, a.r, SB + k);
            if (c.t == 0) {
                double2 n2 = make_double2(0.0, 0.0), cr = make_double2(0.0, 0.0);
                for (int e = 0; e < c.R; ++e) {
                    long i = c.entry(e);
                    cpx<T> z = ck[i], q = a.r[i];
                    n2 = cfma_conj(n2, (double)z.re, (double)z.im, (double)z.re, (double)z.im);
                    cr = cfma_conj(cr, (double)z.re, (double)z.im, (double)q.re, (double)q.im);
                }
                a.part[((long)(SB + 2 * k) * c.G + c.g) * 2] = n2.x;
                a.part[((long)(SB + 2 * k) * c.G + c.g) * 2 + 1] = 0.0;
                a.part[((long)(SB + 2 * k + 1) * c.G + c.g) * 2] = cr.x;
                a.part[((long)(SB + 2 * k + 1) * c.G + c.g) * 2 + 1] = cr.y;
            }
            grid.sync();  // S3
            reduce_slots(a.part, c.G, SB, 2 * k + 2, red);
            // red: [0,k) a2_j; [k,2k) (chi_j, r); 2k: ||chi_k'||^2; 2k+1: (chi_k', r)
            if (c.t == 0) {
                double b2 = red[4 * k];
                double crr = red[4 * k + 2], cri = red[4 * k + 3];
                for (int j = 0; j < k; ++j) {
                    double ar = red[2 * j], ai = red[2 * j + 1];
                    double qr = red[2 * (k + j)], qi = red[2 * (k + j) + 1];
                    b2 -= ar * ar + ai * ai;
                    // (chi_k'', r) = (chi_k', r) - sum conj(a2_j) (chi_j, r)
                    crr -= ar * qr + ai * qi;
                    cri -= ar * qi - ai * qr;
                    acoef[j][k][0] += ar;
                    acoef[j][k][1] += ai;
                }
                double b = b2 > 0.0 ? sqrt(b2) : 0.0;
                bcoef[k] = b;
                ccoef[k][0] = b > 0.0 ? crr / b : 0.0;
                ccoef[k][1] = b > 0.0 ? cri / b : 0.0;
            }
            __syncthreads();
            const double b = bcoef[k];
            if (!(b > 0.0)) {
                broke = true;  // the new direction lies in the span: end the cycle without it
                break;
            }
            const double inv = 1.0 / b, cr0 = ccoef[k][0], ci0 = ccoef[k][1];
            for (int e = c.t; e < c.R; e += LT) {
                long i = c.entry(e);
                double yr = (double)ck[i].re, yi = (double)ck[i].im;
                for (int j = 0; j < k; ++j) {
                    cpx<T> z = a.chi[(long)j * N + i];
                    yr -= red[2 * j] * (double)z.re - red[2 * j + 1] * (double)z.im;
                    yi -= red[2 * j] * (double)z.im + red[2 * j + 1] * (double)z.re;
                }
                yr *= inv;
                yi *= inv;
                ck[i] = cpx<T>{(T)yr, (T)yi};
                double rr = (double)a.r[i].re - (cr0 * yr - ci0 * yi);
                double ri = (double)a.r[i].im - (cr0 * yi + ci0 * yr);
                a.r[i] = cpx<T>{(T)rr, (T)ri};
            }
            ++iters;
            __syncthreads();
        }
        // x += sum alpha_k xi_k, alpha from the triangular system
        if (c.t == 0) {
            for (int i = k - 1; i >= 0; --i) {
                double sr = ccoef[i][0], si = ccoef[i][1];
                for (int j = i + 1; j < k; ++j) {
                    double ar = acoef[i][j][0], ai = acoef[i][j][1];
                    sr -= ar * alpha[j][0] - ai * alpha[j][1];
                    si -= ar * alpha[j][1] + ai * alpha[j][0];
                }
                alpha[i][0] = sr / bcoef[i];
                alpha[i][1] = si / bcoef[i];
            }
        }
        __syncthreads();
        for (int e = c.t; e < c.R; e += LT) {
            long i = c.entry(e);
            double yr = (double)a.x[i].re, yi = (double)a.x[i].im;
            for (int j = 0; j < k; ++j) {
                cpx<T> z = a.xi[(long)j * N + i];
                yr += alpha[j][0] * (double)z.re - alpha[j][1] * (double)z.im;
                yi += alpha[j][0] * (double)z.im + alpha[j][1] * (double)z.re;
            }
            a.x[i] = cpx<T>{(T)yr, (T)yi};
        }
        // recompute r = w - A x
        grid.sync();
        apply_rows(c, a.x, a.r);
        __syncthreads();
        for (int e = c.t; e < c.R; e += LT) {
            long i = c.entry(e);
            a.r[i] = cpx<T>{(T)((double)a.w[i].re - (double)a.r[i].re), (T)((double)a.w[i].im - (double)a.r[i].im)};
        }
        partial_norm2(c, a.r, SR, sh);
        grid.sync();
        reduce_slots(a.part, c.G, SR, 1, red);
        if (c.t == 0)
            rn2_s = red[0];
        __syncthreads();
        converged = rn2_s <= a.tol2 * wn2;
    }
    if (c.g == 0 && c.t == 0) {
        atomicAdd(&a.stats[0], iters);
        atomicAdd(&a.stats[1], 1);
        if (!converged)
            atomicOr(&a.stats[2], 1);
    }
}

template <typename T>
void launch_impl(const Geom& g, int Ns, int nkv, int maxiter, double tol, const cpx<T>* At, const cpx<T>* w,
                 cpx<T>* x, cpx<T>* r, cpx<T>* xi, cpx<T>* chi, double* part, int* stats, int grid_size,
                 hipStream_t s)
{
    LittleArgs<T> a;
    a.g = g;
    a.Ns = Ns;
    a.nkv = nkv;
    a.maxiter = maxiter;
    a.tol2 = tol * tol;
    a.At = At;
    a.w = w;
    a.x = x;
    a.r = r;
    a.xi = xi;
    a.chi = chi;
    a.part = part;
    a.stats = stats;
    void* args[] = {&a};
    HIPCHECK(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_little_gcr<T>), dim3(grid_size), dim3(LT),
                                        args, 0, s));
}

}  // namespace

int little_gcr_grid(const Geom& g)
{
    int G = g.Nb < kLittleMaxGrid ? g.Nb : kLittleMaxGrid;
    return G < 1 ? 1 : G;
}

size_t little_gcr_partial_doubles(int grid_size) { return (size_t)NSLOT * grid_size * 2; }

template <typename T>
void launch_little_gcr(const Geom& g, int Ns, int nkv, int maxiter, double tol, const cpx<T>* At, const cpx<T>* w,
                       cpx<T>* x, cpx<T>* r, cpx<T>* xi, cpx<T>* chi, double* part, int* stats, hipStream_t s)
{
    launch_impl<T>(g, Ns, nkv, maxiter, tol, At, w, x, r, xi, chi, part, stats, little_gcr_grid(g), s);
}

template void launch_little_gcr<double>(const Geom&, int, int, int, double, const c64*, const c64*, c64*, c64*, c64*,
                                        c64*, double*, int*, hipStream_t);
template void launch_little_gcr<float>(const Geom&, int, int, int, double, const c32*, const c32*, c32*, c32*, c32*,
                                       c32*, double*, int*, hipStream_t);

}  // namespace dfl
