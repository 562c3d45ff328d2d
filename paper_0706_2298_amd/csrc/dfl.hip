// Block-projection kernels of the deflation subspace (sections 4.1-4.2 and
// appendix A.1). The deflation blocks are the layout blocks, so every block
// is a contiguous run of Vb sites in each of the 12 planes: one workgroup per
// block reads its block of every basis field with unit stride.
#include "internal.h"

namespace dfl {

namespace {

constexpr int kBT = 256;  // threads per block-kernel workgroup

constexpr int kRB = 8;  // right-hand sides per pass of the batched projections

// Address of the e-th of the 12*Vb entries of block blk in a native field.
// When Vb is a multiple of the 64-site tile, a block is one contiguous run.
__device__ inline long block_elem(const Geom& g, int blk, int e)
{
    if ((g.Vb & (kTile - 1)) == 0)
        return (long)blk * 12 * g.Vb + e;
    const int t = e % g.Vb, c = e / g.Vb;
    return tidx((long)blk * g.Vb + t, c, 12);
}

// w_b[blk*Ns + k] = sum_{x in blk} sum_c conj(Phi_k(x,c)) psi_b(x,c)   (eq. (4.1))
// One workgroup per (block, k); the Ns workgroups of a block are adjacent in
// the XCD-remapped order, so the block of psi_b is fetched into one L2. The
// Phi_k entries are read once per chunk of RB right-hand sides (one pass
// over eight right-hand sides has nine loads per entry in flight). A single
// field uses k_restrict_kg below.
template <int RB, typename P>
__global__ __launch_bounds__(kBT) void k_restrict(Geom g, const P* __restrict__ Phi, int Ns,
                                                  const c64* __restrict__ psi, c64* __restrict__ w, int nrhs,
                                                  int grid_padded)
{
    __shared__ double part[2 * RB][kBT / 64];
    const int q = xcd_remap(blockIdx.x, grid_padded);
    if (q >= g.Nb * Ns)
        return;
    const int blk = q / Ns, k = q - blk * Ns;
    const long fs = 12 * g.V;
    const long nw = (long)g.Nb * Ns;
    const P* ph = Phi + (long)k * fs;
    const int ne = 12 * g.Vb;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int b0 = 0; b0 < nrhs; b0 += RB) {
        double re[RB], im[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j)
            re[j] = im[j] = 0.0;
        for (int e = threadIdx.x; e < ne; e += kBT) {
            const long i = block_elem(g, blk, e);
            const c64 a = c64{(double)ph[i].re, (double)ph[i].im};
#pragma unroll
            for (int j = 0; j < RB; ++j)
                if (b0 + j < nrhs) {
                    const c64 b = psi[(long)(b0 + j) * fs + i];
                    re[j] += a.re * b.re + a.im * b.im;
                    im[j] += a.re * b.im - a.im * b.re;
                }
        }
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            double x = wave_sum(re[j]), y = wave_sum(im[j]);
            if (lane == 0) {
                part[2 * j][wid] = x;
                part[2 * j + 1][wid] = y;
            }
        }
        __syncthreads();
        if (threadIdx.x < 2 * RB && b0 + (threadIdx.x >> 1) < nrhs) {
            double t = 0.0;
            for (int u = 0; u < kBT / 64; ++u)
                t += part[threadIdx.x][u];
            double* dst = reinterpret_cast<double*>(w + (long)(b0 + (threadIdx.x >> 1)) * nw + q);
            dst[threadIdx.x & 1] = t;
        }
        __syncthreads();
    }
}

// Single field, KG basis fields per workgroup: one workgroup per (block,
// group of KG consecutive k); each entry of psi is loaded once for the KG
// products (the block of psi is fetched Ns / KG times instead of Ns).
template <int KG, typename P>
__global__ __launch_bounds__(kBT) void k_restrict_kg(Geom g, const P* __restrict__ Phi, int Ns,
                                                     const c64* __restrict__ psi, c64* __restrict__ w, int ngrp,
                                                     int grid_padded)
{
    __shared__ double part[2 * KG][kBT / 64];
    const int q = xcd_remap(blockIdx.x, grid_padded);
    if (q >= g.Nb * ngrp)
        return;
    const int blk = q / ngrp, k0 = (q - blk * ngrp) * KG;
    const long fs = 12 * g.V;
    const int ne = 12 * g.Vb;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double re[KG], im[KG];
#pragma unroll
    for (int j = 0; j < KG; ++j)
        re[j] = im[j] = 0.0;
    constexpr int RU = 4;
    for (int e0 = threadIdx.x; e0 < ne; e0 += RU * kBT) {
        c64 bv[RU];
        P av[RU][KG];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const long i = block_elem(g, blk, min(e0 + u * kBT, ne - 1));
            bv[u] = psi[i];
#pragma unroll
            for (int j = 0; j < KG; ++j)
                av[u][j] = Phi[(long)min(k0 + j, Ns - 1) * fs + i];
        }
#pragma unroll
        for (int u = 0; u < RU; ++u)
            if (e0 + u * kBT < ne) {
#pragma unroll
                for (int j = 0; j < KG; ++j) {
                    const c64 a = c64{(double)av[u][j].re, (double)av[u][j].im}, b = bv[u];
                    re[j] += a.re * b.re + a.im * b.im;
                    im[j] += a.re * b.im - a.im * b.re;
                }
            }
    }
#pragma unroll
    for (int j = 0; j < KG; ++j) {
        const double x = wave_sum(re[j]), y = wave_sum(im[j]);
        if (lane == 0) {
            part[2 * j][wid] = x;
            part[2 * j + 1][wid] = y;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * KG && k0 + (threadIdx.x >> 1) < Ns) {
        double t = 0.0;
        for (int u = 0; u < kBT / 64; ++u)
            t += part[threadIdx.x][u];
        double* dst = reinterpret_cast<double*>(w + (long)blk * Ns + k0 + (threadIdx.x >> 1));
        dst[threadIdx.x & 1] = t;
    }
}

// psi_b(i) = sum_k Phi_k(i) v_b[blk(i)*Ns + k], one thread per field entry
template <typename P>
__global__ __launch_bounds__(256) void k_prolong(Geom g, const P* __restrict__ Phi, int Ns,
                                                 const c64* __restrict__ v, c64* __restrict__ psi, int nrhs)
{
    const long fs = 12 * g.V;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= fs)
        return;
    const long s = (i / (12 * kTile)) * kTile + (i & (kTile - 1));
    const long blk = s / g.Vb;
    const long nw = (long)g.Nb * Ns;
    for (int b0 = 0; b0 < nrhs; b0 += kRB) {
        c64 acc[kRB];
#pragma unroll
        for (int j = 0; j < kRB; ++j)
            acc[j] = c64{0.0, 0.0};
        for (int k = 0; k < Ns; ++k) {
            const c64 a = c64{(double)Phi[(long)k * fs + i].re, (double)Phi[(long)k * fs + i].im};
#pragma unroll
            for (int j = 0; j < kRB; ++j)
                if (b0 + j < nrhs)
                    acc[j] += a * v[(long)(b0 + j) * nw + blk * Ns + k];
        }
#pragma unroll
        for (int j = 0; j < kRB; ++j)
            if (b0 + j < nrhs)
                psi[(long)(b0 + j) * fs + i] = acc[j];
    }
}

// The same when every 64-site tile lies in one block (Vb a multiple of 64):
// a workgroup's 256 entries are a third of one tile, so the block and its
// coefficients are uniform across the workgroup (scalar loads), and eight
// basis fields' loads are issued together.
template <typename P>
__global__ __launch_bounds__(256) void k_prolong_tile(Geom g, const P* __restrict__ Phi, int Ns,
                                                      const c64* __restrict__ v, c64* __restrict__ psi, int nrhs)
{
    constexpr int KU = 8;
    const long fs = 12 * g.V;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long blk = (long)(blockIdx.x / 3) * kTile / g.Vb;
    const long nw = (long)g.Nb * Ns;
    for (int b0 = 0; b0 < nrhs; b0 += kRB) {
        c64 acc[kRB];
#pragma unroll
        for (int j = 0; j < kRB; ++j)
            acc[j] = c64{0.0, 0.0};
        for (int k0 = 0; k0 < Ns; k0 += KU) {
            c64 a[KU];
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                const int k = min(k0 + u, Ns - 1);  // past Ns: a valid field, weight dropped below
                a[u] = c64{(double)Phi[(long)k * fs + i].re, (double)Phi[(long)k * fs + i].im};
            }
#pragma unroll
            for (int u = 0; u < KU; ++u)
                if (k0 + u < Ns)
#pragma unroll
                    for (int j = 0; j < kRB; ++j)
                        if (b0 + j < nrhs)
                            acc[j] += a[u] * v[(long)(b0 + j) * nw + blk * Ns + k0 + u];
        }
#pragma unroll
        for (int j = 0; j < kRB; ++j)
            if (b0 + j < nrhs)
                psi[(long)(b0 + j) * fs + i] = acc[j];
    }
}

// Modified Gram-Schmidt per block, in place, order l = 0..Ns-1 (eq. (4.2)).
// flag is set to 1 if a block loses rank; R (may be null) receives the
// triangular factor. One workgroup per block; the field being orthogonalised
// is held in registers (E entries per thread, 12 Vb <= E kBT), so each
// projection reads only the earlier basis field and needs one reduction.
// Blocks of more than 512 sites use k_block_gs_stream, which streams both
// fields through memory.

// sum over the workgroup of a complex value, the same in every thread (fixed order)
__device__ inline double2 block_sum2(double2 v, double2* sh)
{
    v.x = wave_sum(v.x);
    v.y = wave_sum(v.y);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0)
        sh[wid] = v;
    __syncthreads();
    double2 t = make_double2(0.0, 0.0);
    for (int q = 0; q < nw; ++q) {
        t.x += sh[q].x;
        t.y += sh[q].y;
    }
    __syncthreads();
    return t;
}

template <int E>
__global__ __launch_bounds__(kBT) void k_block_gs(Geom g, c64* __restrict__ F, int Ns, double rank_tol,
                                                  int* __restrict__ flag, c64* __restrict__ R)
{
    __shared__ double2 sh[kBT / 64];
    const int blk = blockIdx.x;
    const long fs = 12 * g.V;
    const int ne = 12 * g.Vb;
    for (int l = 0; l < Ns; ++l) {
        c64* fl = F + (long)l * fs;
        c64 v[E];
        double n0 = 0.0;
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int e = threadIdx.x + j * kBT;
            v[j] = e < ne ? fl[block_elem(g, blk, e)] : c64{0.0, 0.0};
            n0 += v[j].re * v[j].re + v[j].im * v[j].im;
        }
        // norm of the restricted input field (for the rank test)
        n0 = block_sum2(make_double2(n0, 0.0), sh).x;
        // the next earlier field's entries are loaded before this projection's reduction
        c64 un[E];
        auto load = [&](int k) {
            const c64* fk = F + (long)k * fs;
#pragma unroll
            for (int j = 0; j < E; ++j) {
                const int e = threadIdx.x + j * kBT;
                un[j] = e < ne ? fk[block_elem(g, blk, e)] : c64{0.0, 0.0};
            }
        };
        if (l > 0)
            load(0);
        for (int k = 0; k < l; ++k) {
            c64 u[E];
#pragma unroll
            for (int j = 0; j < E; ++j)
                u[j] = un[j];
            if (k + 1 < l)
                load(k + 1);
            double2 d = make_double2(0.0, 0.0);
#pragma unroll
            for (int j = 0; j < E; ++j) {
                d.x += u[j].re * v[j].re + u[j].im * v[j].im;
                d.y += u[j].re * v[j].im - u[j].im * v[j].re;
            }
            d = block_sum2(d, sh);
            const c64 cf{d.x, d.y};
            if (R && threadIdx.x == 0)
                R[((long)blk * Ns + k) * Ns + l] = cf;
#pragma unroll
            for (int j = 0; j < E; ++j)
                v[j] -= cf * u[j];
        }
        double nv = 0.0;
#pragma unroll
        for (int j = 0; j < E; ++j)
            nv += v[j].re * v[j].re + v[j].im * v[j].im;
        nv = sqrt(block_sum2(make_double2(nv, 0.0), sh).x);
        n0 = sqrt(n0);
        if (R && threadIdx.x == 0) {
            R[((long)blk * Ns + l) * Ns + l] = c64{nv, 0.0};
            for (int k = l + 1; k < Ns; ++k)
                R[((long)blk * Ns + k) * Ns + l] = c64{0.0, 0.0};
        }
        if (!(nv > rank_tol * n0) || !(n0 > 0.0)) {
            if (threadIdx.x == 0)
                atomicOr(flag, 2);
            nv = 1.0;
        }
        const double inv = 1.0 / nv;
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int e = threadIdx.x + j * kBT;
            if (e < ne)
                fl[block_elem(g, blk, e)] = c64{v[j].re * inv, v[j].im * inv};
        }
    }
}

// The same modified Gram-Schmidt with the fields taken G at a time, NT
// threads of E entries each: the G fields of a group are held in registers
// and projected against each earlier basis field in one pass (one load of
// that field and one workgroup sum of the G products), then against each
// other in order. Each field sees the same sequence of projections as in
// k_block_gs; the products of field l with the later fields of its group are
// summed with the norm of l, before l is scaled (the results agree up to that
// rounding). Every earlier basis field is read once per group.
constexpr int kGsGroup = 4;  // fields per group of k_block_gsg on blocks of up to 512 sites
template <int E, int NT, int G>
__global__ __launch_bounds__(NT) void k_block_gsg(Geom g, c64* __restrict__ F, int Ns, double rank_tol,
                                                   int* __restrict__ flag, c64* __restrict__ R, c64* __restrict__ FT,
                                                   c32* __restrict__ F32)
{
    __shared__ double2 sh[2][G][NT / 64];
    const int blk = blockIdx.x;
    const long fs = 12 * g.V;
    const int ne = 12 * g.Vb;
    const bool b4 = g.b[0] == 4 && g.b[1] == 4 && g.b[2] == 4 && g.b[3] == 4;
    // workgroup sums of the first nv (<= G) complex values of v, the same in
    // every thread afterwards. Consecutive sums use alternate LDS slots, so
    // one barrier each suffices: a slot is written again only after the
    // barrier of the next sum, which every thread passes after reading it.
    int par = 0;
    auto sumN = [&](double2* v, int nv) {
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
        for (int q = 0; q < G; ++q)
            if (q < nv) {
                v[q].x = wave_sum(v[q].x);
                v[q].y = wave_sum(v[q].y);
                if (lane == 0)
                    sh[par][q][wid] = v[q];
            }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < G; ++q)
            if (q < nv) {
                double2 t = make_double2(0.0, 0.0);
                for (int w = 0; w < nw; ++w) {
                    t.x += sh[par][q][w].x;
                    t.y += sh[par][q][w].y;
                }
                v[q] = t;
            }
        par ^= 1;
    };
    auto load_field = [&](int k, c64* w) {
        const c64* fk = F + (long)k * fs;
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int e = threadIdx.x + j * NT;
            w[j] = e < ne ? fk[block_elem(g, blk, e)] : c64{0.0, 0.0};
        }
    };
    // normalise v (field l, input norm n0), store it, record the diagonal of
    // R; returns the factor applied
    auto finish = [&](int l, c64* v, double n0, double nv2) -> double {
        double nv = sqrt(nv2);
        n0 = sqrt(n0);
        if (R && threadIdx.x == 0) {
            R[((long)blk * Ns + l) * Ns + l] = c64{nv, 0.0};
            for (int k = l + 1; k < Ns; ++k)
                R[((long)blk * Ns + k) * Ns + l] = c64{0.0, 0.0};
        }
        if (!(nv > rank_tol * n0) || !(n0 > 0.0)) {
            if (threadIdx.x == 0)
                atomicOr(flag, 2);
            nv = 1.0;
        }
        const double inv = 1.0 / nv;
        c64* fl = F + (long)l * fs;
#pragma unroll
        for (int j = 0; j < E; ++j) {
            v[j] = c64{v[j].re * inv, v[j].im * inv};
            const int e = threadIdx.x + j * NT;
            if (e < ne) {
                const long i = block_elem(g, blk, e);
                fl[i] = v[j];
                if (F32)
                    F32[(long)l * fs + i] = c32{(float)v[j].re, (float)v[j].im};
                if (FT) {
                    // the same entry in the transposed in-block order
                    long it;
                    if (b4) {
                        // 4^4 block, entry e = 768 y0 + 64 c + 16 y1 + 4 y2 + y3: the transposed
                        // site has tile y3 and lane 16 y2 + 4 y1 + y0
                        const int y0 = e / (12 * kTile), ln = e & (kTile - 1), c = (e >> 6) % 12;
                        it = (long)blk * ne + (ln & 3) * (12 * kTile) + c * kTile + ((ln >> 2) & 3) * 16 +
                             (ln >> 4) * 4 + y0;
                    } else {
                        const long st = (i / (12 * kTile)) * kTile + (i & (kTile - 1));
                        int n[4], y[4];
                        site_decompose(g, st, n, y);
                        it = tidx(site_compose_t(g, n, y), (int)((i / kTile) % 12), 12);
                    }
                    FT[(long)l * fs + it] = v[j];
                }
            }
        }
        return inv;
    };
    for (int l0 = 0; l0 < Ns; l0 += G) {
        const int cnt = min(G, Ns - l0);
        c64 v[G][E];
        double2 s[G];
#pragma unroll
        for (int f = 0; f < G; ++f) {
            if (f < cnt)
                load_field(l0 + f, v[f]);
            else
#pragma unroll
                for (int j = 0; j < E; ++j)
                    v[f][j] = c64{0.0, 0.0};
        }
        // input norms (the reference of the rank test)
#pragma unroll
        for (int f = 0; f < G; ++f) {
            s[f] = make_double2(0.0, 0.0);
#pragma unroll
            for (int j = 0; j < E; ++j)
                s[f].x += v[f][j].re * v[f][j].re + v[f][j].im * v[f][j].im;
        }
        sumN(s, G);
        double n0[G];
#pragma unroll
        for (int f = 0; f < G; ++f)
            n0[f] = s[f].x;
        // against the earlier basis fields, the next one's load issued ahead
        c64 un[E];
        if (l0 > 0)
            load_field(0, un);
        for (int k = 0; k < l0; ++k) {
            c64 u[E];
#pragma unroll
            for (int j = 0; j < E; ++j)
                u[j] = un[j];
            if (k + 1 < l0)
                load_field(k + 1, un);
#pragma unroll
            for (int f = 0; f < G; ++f) {
                s[f] = make_double2(0.0, 0.0);
#pragma unroll
                for (int j = 0; j < E; ++j) {
                    s[f].x += u[j].re * v[f][j].re + u[j].im * v[f][j].im;
                    s[f].y += u[j].re * v[f][j].im - u[j].im * v[f][j].re;
                }
            }
            sumN(s, G);
            if (R && threadIdx.x == 0) {
#pragma unroll
                for (int f = 0; f < G; ++f)
                    if (f < cnt)
                        R[((long)blk * Ns + k) * Ns + l0 + f] = c64{s[f].x, s[f].y};
            }
#pragma unroll
            for (int f = 0; f < G; ++f) {
                const c64 c{s[f].x, s[f].y};
#pragma unroll
                for (int j = 0; j < E; ++j)
                    v[f][j] -= c * u[j];
            }
        }
        // within the group, in order: the norm of field f and its products
        // with the later fields in one sum, then f is scaled and stored and
        // the later fields continue against it
#pragma unroll
        for (int f = 0; f < G; ++f) {
            if (f >= cnt)
                break;
#pragma unroll
            for (int h = 0; h < G; ++h) {
                s[h] = make_double2(0.0, 0.0);
                if (h == 0) {
#pragma unroll
                    for (int j = 0; j < E; ++j)
                        s[0].x += v[f][j].re * v[f][j].re + v[f][j].im * v[f][j].im;
                } else if (f + h < G) {
#pragma unroll
                    for (int j = 0; j < E; ++j) {
                        s[h].x += v[f][j].re * v[f + h][j].re + v[f][j].im * v[f + h][j].im;
                        s[h].y += v[f][j].re * v[f + h][j].im - v[f][j].im * v[f + h][j].re;
                    }
                }
            }
            sumN(s, cnt - f);
            const double inv = finish(l0 + f, v[f], n0[f], s[0].x);
#pragma unroll
            for (int h = 1; h < G; ++h) {
                if (f + h < cnt) {
                    const c64 c{s[h].x * inv, s[h].y * inv};
                    if (R && threadIdx.x == 0)
                        R[((long)blk * Ns + l0 + f) * Ns + l0 + f + h] = c;
#pragma unroll
                    for (int j = 0; j < E; ++j)
                        v[f + h][j] -= c * v[f][j];
                }
            }
        }
    }
}

// The same Gram-Schmidt for blocks of any size, both fields streamed through memory.
__global__ __launch_bounds__(kBT) void k_block_gs_stream(Geom g, c64* __restrict__ F, int Ns, double rank_tol,
                                                  int* __restrict__ flag, c64* __restrict__ R)
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
            if (R && threadIdx.x == 0)
                R[((long)blockIdx.x * Ns + k) * Ns + l] = cf;
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
        if (R && threadIdx.x == 0) {
            R[((long)blockIdx.x * Ns + l) * Ns + l] = c64{nv, 0.0};
            for (int k = l + 1; k < Ns; ++k)
                R[((long)blockIdx.x * Ns + k) * Ns + l] = c64{0.0, 0.0};
        }
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

// index of the d-th neighbour of block blk (d = 0 itself, 1 + 2mu: +mu, 2 + 2mu: -mu)
__device__ inline int block_nbr(const Geom& g, int blk, int d)
{
    if (d == 0)
        return blk;
    const int mu = (d - 1) >> 1;
    int rest = blk;
    for (int nu = 3; nu > mu; --nu)
        rest /= g.nb[nu];
    const int n_mu = rest % g.nb[mu];
    int nn = n_mu + ((d & 1) ? 1 : -1);
    if (nn < 0)
        nn += g.nb[mu];
    if (nn >= g.nb[mu])
        nn -= g.nb[mu];
    return blk + (nn - n_mu) * g.bstr[mu];
}

// Block products Phi_blk^+ Y_blk of eq. (A.1) for nc columns at once, the
// 12 Vb entries of a block split over nsplit workgroups:
// part[split][blk][k][j] = sum over the split's entries of conj(Phi_k) Y_j.
// Entries are staged through LDS kCE at a time, each thread accumulating up
// to kMaxPairs of the Ns*nc products.
constexpr int kCE = 32;
constexpr int kMaxPairs = 16;

// Entry e of the block's face {y_fmu = fy} (fmu >= 0; e = c * nface + site
// index in local lexicographic order) or of the whole block (fmu < 0).
__device__ inline long face_elem(const Geom& g, int blk, int e, int fmu, int fy, int nface)
{
    if (fmu < 0)
        return block_elem(g, blk, e);
    const int c = e / nface;
    int r = e - c * nface, y[4];
#pragma unroll
    for (int nu = 3; nu >= 0; --nu) {
        if (nu == fmu) {
            y[nu] = fy;
        } else {
            y[nu] = r % g.b[nu];
            r /= g.b[nu];
        }
    }
    const int t = ((y[0] * g.b[1] + y[1]) * g.b[2] + y[2]) * g.b[3] + y[3];
    return tidx((long)blk * g.Vb + t, c, 12);
}

// The same for fields stored in the transposed in-block order (y0 fastest;
// site_compose_t), the face sites enumerated in that order.
__device__ inline long face_elem_t(const Geom& g, int blk, int e, int fmu, int fy, int nface)
{
    const int c = e / nface;
    int r = e - c * nface, y[4];
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == fmu) {
            y[nu] = fy;
        } else {
            y[nu] = r % g.b[nu];
            r /= g.b[nu];
        }
    }
    const int t = ((y[3] * g.b[2] + y[2]) * g.b[1] + y[1]) * g.b[0] + y[0];
    return tidx((long)blk * g.Vb + t, c, 12);
}

// A block hop (eq. (A.1) with D restricted to the hops from block Lambda + mu
// into Lambda) is non-zero only on the sites of Lambda's face towards
// Lambda + mu: for those columns only that face's entries are summed.
__global__ __launch_bounds__(256) void k_little_columns(Geom g, const c64* __restrict__ Phi, int Ns,
                                                        const c64* __restrict__ Y, int nc, int nsplit, int fmu,
                                                        int fy, int nface, c64* __restrict__ part)
{
    extern __shared__ c64 st[];  // [Ns + nc][kCE + 1]
    __shared__ long eidx[kCE];
    const int blk = blockIdx.x / nsplit, split = blockIdx.x % nsplit;
    const long F = 12 * g.V;
    const int ne = 12 * nface;  // nface: sites of the face (Vb for the whole block)
    const int per = ((ne + nsplit - 1) / nsplit + kCE - 1) / kCE * kCE;
    const int e_lo = split * per;
    const int e_hi = e_lo + per < ne ? e_lo + per : ne;
    const int np = Ns * nc;
    c64 acc[kMaxPairs];
#pragma unroll
    for (int q = 0; q < kMaxPairs; ++q)
        acc[q] = c64{0.0, 0.0};
    for (int e0 = e_lo; e0 < e_hi; e0 += kCE) {
        __syncthreads();
        if (threadIdx.x < kCE)
            eidx[threadIdx.x] = e0 + (int)threadIdx.x < e_hi ? face_elem(g, blk, e0 + threadIdx.x, fmu, fy, nface) : -1;
        __syncthreads();
        for (int q = threadIdx.x; q < (Ns + nc) * kCE; q += blockDim.x) {
            const int r = q / kCE, e = q % kCE;
            c64 v{0.0, 0.0};
            const long i = eidx[e];
            if (i >= 0)
                v = r < Ns ? Phi[(long)r * F + i] : Y[(long)(r - Ns) * F + i];
            st[r * (kCE + 1) + e] = v;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kMaxPairs; ++q) {
            const int p = threadIdx.x + q * blockDim.x;
            if (p < np) {
                const int k = p / nc, j = p - k * nc;
                const c64* u = st + k * (kCE + 1);
                const c64* v = st + (Ns + j) * (kCE + 1);
                double re = acc[q].re, im = acc[q].im;
                for (int e = 0; e < kCE; ++e) {
                    const c64 a = u[e], b = v[e];
                    re += a.re * b.re + a.im * b.im;
                    im += a.re * b.im - a.im * b.re;
                }
                acc[q] = c64{re, im};
            }
        }
    }
#pragma unroll
    for (int q = 0; q < kMaxPairs; ++q) {
        const int p = threadIdx.x + q * blockDim.x;
        if (p < np)
            part[((long)split * g.Nb + blk) * np + p] = acc[q];
    }
}

// Register-tiled form for Ns <= 4 TK and nc <= 16: the (k, j) pairs form 16
// tiles of TK x 4, one per 16-lane row of the workgroup; the 16 lanes of a
// row take every 16th staged entry, read TK + 4 values from LDS per entry for
// 4 TK products (the kernel above reads 2 per product), and combine their
// sums with in-row DPP moves at the end. Same partial-sum layout as above.
// TK = 5 serves Ns <= 20, TK = 6 Ns <= 24.
constexpr int kRtJ = 4, kRtCE = 64;

__device__ inline double row16_sum(double v)
{
    using namespace wave_detail;
    v += dpp<0xB1, 0xF>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp<0x4E, 0xF>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp<0x141, 0xF>(v);  // row_half_mirror
    v += dpp<0x140, 0xF>(v);  // row_mirror
    return v;
}

template <int TK, bool TL>
__global__ __launch_bounds__(256) void k_little_columns_rt(Geom g, const c64* __restrict__ Phi, int Ns,
                                                           const c64* __restrict__ Y, int nc, int nsplit, int fmu,
                                                           int fy, int nface, c64* __restrict__ part)
{
    constexpr int kRtK = TK;
    constexpr int kRtLd = (4 * kRtK + 4 * kRtJ + 3) / 4;  // staged rows per thread (Ns + nc rows over 4 waves)
    extern __shared__ c64 st[];  // [Ns + nc][kRtCE]
    const int blk = blockIdx.x / nsplit, split = blockIdx.x % nsplit;
    const long F = 12 * g.V;
    const int ne = 12 * nface;
    const int per = ((ne + nsplit - 1) / nsplit + kRtCE - 1) / kRtCE * kRtCE;
    const int e_lo = split * per;
    const int e_hi = e_lo + per < ne ? e_lo + per : ne;
    const int nr = Ns + nc;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int lane16 = threadIdx.x & 15, tile = threadIdx.x >> 4;
    const int k0 = (tile >> 2) * kRtK, j0 = (tile & 3) * kRtJ;
    double acc[kRtK][kRtJ][2];
#pragma unroll
    for (int i = 0; i < kRtK; ++i)
#pragma unroll
        for (int j = 0; j < kRtJ; ++j)
            acc[i][j][0] = acc[i][j][1] = 0.0;
    // staging: entry e0 + lane of rows wid, wid + 4, ... (kRtCE = 64 entries,
    // 256 threads), all loads of a stage issued together, the next stage's
    // during the current stage's products
    c64 v[kRtLd];
    auto load = [&](int e0) {
        const long i = e0 + lane >= e_hi ? -1
                       : (TL ? face_elem_t(g, blk, e0 + lane, fmu, fy, nface)
                             : face_elem(g, blk, e0 + lane, fmu, fy, nface));
#pragma unroll
        for (int m = 0; m < kRtLd; ++m) {
            const int r = wid + 4 * m;
            v[m] = c64{0.0, 0.0};
            if (i >= 0 && r < nr)
                v[m] = r < Ns ? Phi[(long)r * F + i] : Y[(long)(r - Ns) * F + i];
        }
    };
    if (e_lo < e_hi)
        load(e_lo);
    for (int e0 = e_lo; e0 < e_hi; e0 += kRtCE) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kRtLd; ++m) {
            const int r = wid + 4 * m;
            if (r < nr)
                st[r * kRtCE + lane] = v[m];
        }
        __syncthreads();
        if (e0 + kRtCE < e_hi)
            load(e0 + kRtCE);
        for (int e = lane16; e < kRtCE; e += 16) {
            c64 a[kRtK], b[kRtJ];
#pragma unroll
            for (int i = 0; i < kRtK; ++i)
                a[i] = k0 + i < Ns ? st[(k0 + i) * kRtCE + e] : c64{0.0, 0.0};
#pragma unroll
            for (int j = 0; j < kRtJ; ++j)
                b[j] = j0 + j < nc ? st[(Ns + j0 + j) * kRtCE + e] : c64{0.0, 0.0};
#pragma unroll
            for (int i = 0; i < kRtK; ++i)
#pragma unroll
                for (int j = 0; j < kRtJ; ++j) {
                    acc[i][j][0] += a[i].re * b[j].re + a[i].im * b[j].im;
                    acc[i][j][1] += a[i].re * b[j].im - a[i].im * b[j].re;
                }
        }
    }
    const int np = Ns * nc;
#pragma unroll
    for (int i = 0; i < kRtK; ++i)
#pragma unroll
        for (int j = 0; j < kRtJ; ++j) {
            const double re = row16_sum(acc[i][j][0]), im = row16_sum(acc[i][j][1]);
            if (lane16 == 0 && k0 + i < Ns && j0 + j < nc)
                part[((long)split * g.Nb + blk) * np + (k0 + i) * nc + j0 + j] = c64{re, im};
        }
}

// Matrix-core form for all Ns columns of a direction at once (Ns <= 32), so
// that the block of every basis field is read once per direction. The
// complex products C[k][j] = sum_e conj(Phi_k(e)) Y_j(e) are the real
// product P Q over two real K indices per entry (the parts of Y_j(e) it
// multiplies): P[2k][.] = (Re Phi_k, Im Phi_k), P[2k+1][.] = (-Im Phi_k,
// Re Phi_k), Q[.][j] = (Re Y_j, Im Y_j). It runs as 16x16x4 FP64 MFMA tiles,
// RT = ceil(2Ns / 16) row tiles by CT = ceil(Ns / 16) column tiles; a pair of
// MFMA steps covers four entries, lane (n, q) supplying Phi_{k(n)}(e0 + q) and
// Y_{j(n)}(e0 + q), their real parts in the first step and their imaginary
// parts in the second. Entries are staged through LDS 64 at a time (rows
// padded to 65 entries); each of the four wavefronts takes 16 of them, and
// the wavefronts' tiles are summed through LDS at the end. Columns
// j < n1 are read from Y1, the others from Y2 (two column buffers). Same
// partial-sum layout as above with nc = Ns.
using f64x4 = __attribute__((ext_vector_type(4))) double;
constexpr int kMfCE = 64;       // entries per stage
constexpr int kColsMinGrid = 2048;  // workgroups of a launch below which a block's entries are split
constexpr int kMfRow = kMfCE + 1;  // staged row stride (entries)

template <int RT, int CT, bool TL>
__global__ __launch_bounds__(256) void k_little_columns_mfma(Geom g, const c64* __restrict__ Phi, int Ns,
                                                             const c64* __restrict__ Y1, int n1,
                                                             const c64* __restrict__ Y2, int nsplit, int fmu, int fy,
                                                             int nface, c64* __restrict__ part)
{
    constexpr int kLd = (16 * RT + 3) / 4;  // staged rows per thread: 2 Ns <= 16 RT rows over 4 wavefronts
    extern __shared__ c64 st[];             // [2 Ns][kMfRow], then the wavefronts' tiles
    const int blk = blockIdx.x / nsplit, split = blockIdx.x % nsplit;
    const long F = 12 * g.V;
    const int ne = 12 * nface;
    const int per = ((ne + nsplit - 1) / nsplit + kMfCE - 1) / kMfCE * kMfCE;
    const int e_lo = split * per;
    const int e_hi = e_lo + per < ne ? e_lo + per : ne;
    const int nr = 2 * Ns;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int n = lane & 15, q = lane >> 4;
    f64x4 acc[RT][CT];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c)
            acc[t][c] = f64x4{0.0, 0.0, 0.0, 0.0};
    c64 v[kLd];
    auto load = [&](int e0) {
        const long i = e0 + lane >= e_hi ? -1
                       : (TL ? face_elem_t(g, blk, e0 + lane, fmu, fy, nface)
                             : face_elem(g, blk, e0 + lane, fmu, fy, nface));
#pragma unroll
        for (int m = 0; m < kLd; ++m) {
            const int r = wid + 4 * m;
            v[m] = c64{0.0, 0.0};
            if (i >= 0 && r < nr) {
                const int j = r - Ns;
                v[m] = r < Ns ? Phi[(long)r * F + i] : (j < n1 ? Y1[(long)j * F + i] : Y2[(long)(j - n1) * F + i]);
            }
        }
    };
    if (e_lo < e_hi)
        load(e_lo);
    for (int e0 = e_lo; e0 < e_hi; e0 += kMfCE) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kLd; ++m) {
            const int r = wid + 4 * m;
            if (r < nr)
                st[r * kMfRow + lane] = v[m];
        }
        __syncthreads();
        if (e0 + kMfCE < e_hi)
            load(e0 + kMfCE);
#pragma unroll
        for (int g4 = 0; g4 < 4; ++g4) {
            const int e = 16 * wid + 4 * g4 + q;
            c64 a[RT], b[CT];
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const int k = 8 * t + (n >> 1);
                a[t] = k < Ns ? st[k * kMfRow + e] : c64{0.0, 0.0};
            }
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const int j = 16 * c + n;
                b[c] = j < Ns ? st[(Ns + j) * kMfRow + e] : c64{0.0, 0.0};
            }
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                // rows 2k (real part of the product) and 2k + 1 (imaginary part)
                const double p1 = (n & 1) ? -a[t].im : a[t].re;
                const double p2 = (n & 1) ? a[t].re : a[t].im;
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    acc[t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(p1, b[c].re, acc[t][c], 0, 0, 0);
                    acc[t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(p2, b[c].im, acc[t][c], 0, 0, 0);
                }
            }
        }
    }
    // the four wavefronts' tiles, summed in a fixed order: tile element i of
    // lane (n, q) is row 16 t + 4 i + q, column 16 c + n
    __syncthreads();
    double* red = reinterpret_cast<double*>(st);  // [wave][t][c][i][lane]
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                red[(((wid * RT + t) * CT + c) * 4 + i) * 64 + lane] = acc[t][c][i];
    __syncthreads();
    const int np = Ns * Ns;
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
        const int k = p / Ns, j = p - k * Ns;
        double z[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = 2 * k + h;
            const int t = row >> 4, i = (row & 15) >> 2, qq = row & 3;
            const int c = j >> 4, ln = qq * 16 + (j & 15);
            double sum = 0.0;
            for (int w = 0; w < 4; ++w)
                sum += red[(((w * RT + t) * CT + c) * 4 + i) * 64 + ln];
            z[h] = sum;
        }
        part[((long)split * g.Nb + blk) * np + p] = c64{z[0], z[1]};
    }
}

// A[blk][d][k][l0 + j] = sum over splits of part (fixed order)
__global__ __launch_bounds__(256) void k_little_columns_sum(Geom g, const c64* __restrict__ part, int Ns, int nc,
                                                            int nsplit, int l0, int d, c64* __restrict__ A)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int np = Ns * nc;
    if (q >= (long)g.Nb * np)
        return;
    const int blk = (int)(q / np), p = (int)(q - (long)blk * np);
    const int k = p / nc, j = p - k * nc;
    c64 s{0.0, 0.0};
    for (int sp = 0; sp < nsplit; ++sp)
        s += part[((long)sp * g.Nb + blk) * np + p];
    A[(((long)blk * 9 + d) * Ns + k) * Ns + l0 + j] = s;
}

// w_b[blk] = sum_d A[blk][d] v_b[nbr_d(blk)], one thread per (blk, k) row,
// blockIdx.y = right-hand side b (little vectors of Nb*Ns entries, back to back)
template <typename T>
__global__ __launch_bounds__(256) void k_little_apply(Geom g, const cpx<T>* __restrict__ A, int Ns,
                                                      const cpx<T>* __restrict__ v, cpx<T>* __restrict__ w)
{
    const long nw = (long)g.Nb * Ns;
    long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= nw)
        return;
    v += blockIdx.y * nw;
    w += blockIdx.y * nw;
    int blk = (int)(row / Ns);
    int k = (int)(row - (long)blk * Ns);
    double re = 0.0, im = 0.0;
    for (int d = 0; d < 9; ++d) {
        const int nbr = block_nbr(g, blk, d);
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

// Batched FP32 little apply on the matrix cores. For one block the complex
// product Y = sum_d A_d V_d (A_d: Ns x Ns, V_d: Ns x nrhs, the right-hand
// sides' entries on the d-th neighbour block) is the real product of the
// 2Ns x 18Ns matrix with entries Re/Im of A_d arranged as [[ar, -ai],[ai, ar]]
// per complex entry (rows and columns interleaved re/im) and the 18Ns x nrhs
// matrix of the V_d entries read as reals. It runs as 16x16x4 FP32 MFMA
// tiles: wave t of the workgroup owns rows [16t, 16t + 16) of the real
// product, 16 right-hand sides per pass. The V_d entries of the pass are
// staged in LDS as [d][l][b] complex.
constexpr int kMfmaRhs = 16;

__global__ __launch_bounds__(256) void k_little_apply_mfma(Geom g, const c32* __restrict__ At, int Ns,
                                                           const c32* __restrict__ v, c32* __restrict__ w, int nrhs)
{
    extern __shared__ c32 vs[];  // [9][Ns][kMfmaRhs]
    const long nw = (long)g.Nb * Ns;
    const int blk = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m_tiles = (2 * Ns + 15) / 16;
    const int n = lane & 15, kq = lane >> 4;
    const c32* Ab = At + (long)blk * 9 * Ns * Ns;  // [d][l][k] = A[d][k][l]
    for (int b0 = 0; b0 < nrhs; b0 += kMfmaRhs) {
        __syncthreads();
        for (int e = threadIdx.x; e < 9 * Ns * kMfmaRhs; e += blockDim.x) {
            const int b = e % kMfmaRhs;
            const int dl = e / kMfmaRhs;
            const int d = dl / Ns, l = dl - d * Ns;
            c32 x{0.f, 0.f};
            if (b0 + b < nrhs)
                x = v[(long)(b0 + b) * nw + (long)block_nbr(g, blk, d) * Ns + l];
            vs[e] = x;
        }
        __syncthreads();
        for (int t = wave; t < m_tiles; t += blockDim.x / 64) {
            const int rr = 16 * t + n;  // real row of the A operand held by this lane
            const int m = rr >> 1, cr = rr & 1;
            __attribute__((ext_vector_type(4))) float acc = {0.f, 0.f, 0.f, 0.f};
            for (int d = 0; d < 9; ++d) {
                const c32* Ad = Ab + (long)d * Ns * Ns;
                for (int kc = 0; kc < 2 * Ns; kc += 4) {
                    const int kk = kc + kq;  // real column index of the contraction
                    const int l = kk >> 1, ck = kk & 1;
                    float a = 0.f, bv = 0.f;
                    if (kk < 2 * Ns) {
                        if (m < Ns) {
                            const c32 z = Ad[(long)l * Ns + m];
                            a = cr == 0 ? (ck == 0 ? z.re : -z.im) : (ck == 0 ? z.im : z.re);
                        }
                        const c32 y = vs[(d * Ns + l) * kMfmaRhs + n];
                        bv = ck == 0 ? y.re : y.im;
                    }
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc, 0, 0, 0);
                }
            }
            // lane holds rows 16t + 4*(lane/16) + i, column n
            if (b0 + n < nrhs) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int ro = 16 * t + 4 * kq + i;
                    if (ro < 2 * Ns) {
                        float* dst = reinterpret_cast<float*>(w + (long)(b0 + n) * nw + (long)blk * Ns + (ro >> 1));
                        dst[ro & 1] = acc[i];
                    }
                }
            }
        }
    }
}

// Even-odd preparation for one block per workgroup: Gauss-Jordan inversion of
// the diagonal block A[blk][0] with partial pivoting in LDS ([Ns][2 Ns]
// augmented matrix), then M_d = D^-1 A[blk][d], d = 1..8. Output transposed:
// Mt[blk][0][l][k] = D^-1[k][l], Mt[blk][d][l][k] = M_d[k][l].
__global__ __launch_bounds__(256) void k_little_eo_prep(Geom g, const c64* __restrict__ A, int Ns,
                                                        c64* __restrict__ Mt64, c32* __restrict__ Mt32,
                                                        int* __restrict__ flag)
{
    extern __shared__ c64 aug[];  // [Ns][2 Ns], then fcol[Ns]
    c64* fcol = aug + 2 * Ns * Ns;
    __shared__ double sh[16];
    __shared__ int piv_s;
    const int blk = blockIdx.x;
    const int W = 2 * Ns;
    const c64* D = A + (long)blk * 9 * Ns * Ns;
    double amax = 0.0;
    for (int q = threadIdx.x; q < Ns * W; q += blockDim.x) {
        const int i = q / W, j = q % W;
        c64 v{0.0, 0.0};
        if (j < Ns) {
            v = D[i * Ns + j];
            amax = fmax(amax, fabs(v.re) + fabs(v.im));
        } else if (j - Ns == i) {
            v = c64{1.0, 0.0};
        }
        aug[q] = v;
    }
    // largest |re| + |im| of the block (shuffles, then LDS)
    for (int off = 32; off >= 1; off >>= 1)
        amax = fmax(amax, __shfl_xor(amax, off, 64));
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = amax;
    __syncthreads();
    amax = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q)
        amax = fmax(amax, sh[q]);
    for (int col = 0; col < Ns; ++col) {
        if (threadIdx.x == 0) {
            int p = col;
            double best = -1.0;
            for (int i = col; i < Ns; ++i) {
                const c64 v = aug[i * W + col];
                const double m = fabs(v.re) + fabs(v.im);
                if (m > best) {
                    best = m;
                    p = i;
                }
            }
            if (!(best >= 1e-8 * amax))
                atomicOr(flag, 1);
            piv_s = p;
        }
        __syncthreads();
        const int p = piv_s;
        if (p != col)
            for (int j = threadIdx.x; j < W; j += blockDim.x) {
                const c64 t = aug[col * W + j];
                aug[col * W + j] = aug[p * W + j];
                aug[p * W + j] = t;
            }
        __syncthreads();
        const c64 pv = aug[col * W + col];
        const double den = pv.re * pv.re + pv.im * pv.im;
        const c64 inv = den > 0.0 ? c64{pv.re / den, -pv.im / den} : c64{0.0, 0.0};
        __syncthreads();
        for (int j = threadIdx.x; j < W; j += blockDim.x)
            aug[col * W + j] = aug[col * W + j] * inv;
        __syncthreads();
        for (int i = threadIdx.x; i < Ns; i += blockDim.x)
            fcol[i] = aug[i * W + col];
        __syncthreads();
        for (int q = threadIdx.x; q < Ns * W; q += blockDim.x) {
            const int i = q / W, j = q % W;
            if (i != col)
                aug[q] -= fcol[i] * aug[col * W + j];
        }
        __syncthreads();
    }
    // D^-1 = aug[:, Ns:2Ns]
    const long base = (long)blk * 9 * Ns * Ns;
    for (int q = threadIdx.x; q < Ns * Ns; q += blockDim.x) {
        const int k = q / Ns, l = q % Ns;
        const c64 v = aug[k * W + Ns + l];
        Mt64[base + (long)l * Ns + k] = v;
        Mt32[base + (long)l * Ns + k] = c32{(float)v.re, (float)v.im};
    }
    for (int q = threadIdx.x; q < 8 * Ns * Ns; q += blockDim.x) {
        const int d = 1 + q / (Ns * Ns);
        const int rem = q % (Ns * Ns);
        const int k = rem / Ns, l = rem % Ns;
        const c64* Ad = A + ((long)blk * 9 + d) * Ns * Ns;
        double re = 0.0, im = 0.0;
        for (int m = 0; m < Ns; ++m) {
            const c64 a = aug[k * W + Ns + m], b = Ad[(long)m * Ns + l];
            re += a.re * b.re - a.im * b.im;
            im += a.re * b.im + a.im * b.re;
        }
        const long o = base + (long)d * Ns * Ns + (long)l * Ns + k;
        Mt64[o] = c64{re, im};
        Mt32[o] = c32{(float)re, (float)im};
    }
}

// Global modes of the little system (appendix A.3): u_l = the l-th start
// field in the block basis, kept on even blocks: u_l[blk][k] = R[blk][k][l]
// (the block Gram-Schmidt coefficients, psi_l = sum_k R_kl phi_k on each
// block), zero on odd blocks.
__global__ void k_global_modes(Geom g, const c64* __restrict__ R, int Ns, c64* __restrict__ U)
{
    const long N = (long)g.Nb * Ns;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N * Ns)
        return;
    const int l = (int)(q / N);
    const long i = q - (long)l * N;
    const int blk = (int)(i / Ns), k = (int)(i - (long)blk * Ns);
    int sum = 0, rest = blk;
    for (int mu = 3; mu >= 0; --mu) {
        sum += rest % g.nb[mu];
        rest /= g.nb[mu];
    }
    U[q] = (sum & 1) ? c64{0.0, 0.0} : R[((long)blk * Ns + k) * Ns + l];
}

// One even-odd hop for nv little vectors (stride N): on the blocks of the
// given parity, out = alpha s + beta sum_{d=1..8} M_d in_{nbr_d} with the
// transposed matrices Mt of the even-odd preparation; other blocks untouched.
__global__ void k_eo_hop(Geom g, const c64* __restrict__ Mt, int Ns, const c64* __restrict__ in,
                         const c64* __restrict__ sv, c64* __restrict__ out, int parity, double alpha, double beta)
{
    const long N = (long)g.Nb * Ns;
    const long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= N)
        return;
    in += blockIdx.y * N;
    out += blockIdx.y * N;
    if (sv)
        sv += blockIdx.y * N;
    const int blk = (int)(row / Ns), k = (int)(row - (long)blk * Ns);
    int n[4], rest = blk, sum = 0;
    for (int mu = 3; mu >= 0; --mu) {
        n[mu] = rest % g.nb[mu];
        rest /= g.nb[mu];
        sum += n[mu];
    }
    if ((sum & 1) != parity)
        return;
    double re = 0.0, im = 0.0;
    for (int d = 1; d < 9; ++d) {
        const int nbr = block_nbr(g, blk, d);
        const c64* M = Mt + ((long)blk * 9 + d) * Ns * Ns + k;
        const c64* x = in + (long)nbr * Ns;
        // ten terms' loads issued together
#pragma unroll 10
        for (int l = 0; l < Ns; ++l) {
            const c64 p = M[(long)l * Ns], q = x[l];
            re += p.re * q.re - p.im * q.im;
            im += p.re * q.im + p.im * q.re;
        }
    }
    double yr = beta * re, yi = beta * im;
    if (sv) {
        yr += alpha * sv[row].re;
        yi += alpha * sv[row].im;
    }
    out[row] = c64{yr, yi};
}

// G[k][l] = (X_k, X_l) for nv vectors of n entries, one workgroup per pair (fixed order)
__global__ __launch_bounds__(256) void k_gram(const c64* __restrict__ X, long n, int nv, c64* __restrict__ G)
{
    __shared__ double sh[16];
    const int k = blockIdx.x / nv, l = blockIdx.x % nv;
    const c64* a = X + (long)k * n;
    const c64* b = X + (long)l * n;
    double re = 0.0, im = 0.0;
    for (long i = threadIdx.x; i < n; i += blockDim.x) {
        const c64 u = a[i], v = b[i];
        re += u.re * v.re + u.im * v.im;
        im += u.re * v.im - u.im * v.re;
    }
    re = block_sum(re, sh);
    im = block_sum(im, sh);
    if (threadIdx.x == 0)
        G[blockIdx.x] = c64{re, im};
}

// G[k][l] = (X_k, Y_l) for nv vectors each
__global__ __launch_bounds__(256) void k_gram2(const c64* __restrict__ X, const c64* __restrict__ Y, long n, int nv,
                                               c64* __restrict__ G)
{
    __shared__ double sh[16];
    const int k = blockIdx.x / nv, l = blockIdx.x % nv;
    const c64* a = X + (long)k * n;
    const c64* b = Y + (long)l * n;
    double re = 0.0, im = 0.0;
    for (long i = threadIdx.x; i < n; i += blockDim.x) {
        const c64 u = a[i], v = b[i];
        re += u.re * v.re + u.im * v.im;
        im += u.re * v.im - u.im * v.re;
    }
    re = block_sum(re, sh);
    im = block_sum(im, sh);
    if (threadIdx.x == 0)
        G[blockIdx.x] = c64{re, im};
}

// Y_l = sum_k X_k C[k][l], l < m, for nv vectors of n entries (C complex nv x m, device)
__global__ void k_combine(const c64* __restrict__ X, long n, int nv, int m, const c64* __restrict__ C,
                          c64* __restrict__ Y)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int l = blockIdx.y;
    c64 s{0.0, 0.0};
    for (int k = 0; k < nv; ++k)
        s += X[(long)k * n + i] * C[(long)k * m + l];
    Y[(long)l * n + i] = s;
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

template <typename P>
void restrict_any(const Geom& g, const P* Phi, int Ns, const c64* psi, c64* w, int nrhs, hipStream_t s)
{
    const int gp = pad_grid((long)g.Nb * Ns);
    if (nrhs == 1) {
        constexpr int KG = 4;  // measured: five fields per workgroup are no faster
        const int ngrp = (Ns + KG - 1) / KG;
        const int gk = pad_grid((long)g.Nb * ngrp);
        hipLaunchKernelGGL((k_restrict_kg<KG, P>), dim3(gk), dim3(kBT), 0, s, g, Phi, Ns, psi, w, ngrp, gk);
    }
    else
        hipLaunchKernelGGL((k_restrict<kRB, P>), dim3(gp), dim3(kBT), 0, s, g, Phi, Ns, psi, w, nrhs, gp);
}
template <typename P>
void prolong_any(const Geom& g, const P* Phi, int Ns, const c64* v, c64* psi, int nrhs, hipStream_t s)
{
    const long n = 12 * g.V;
    if (g.Vb % kTile == 0)  // then n is a multiple of 3 * 256
        hipLaunchKernelGGL(k_prolong_tile<P>, dim3((unsigned)(n / 256)), dim3(256), 0, s, g, Phi, Ns, v, psi, nrhs);
    else
        hipLaunchKernelGGL(k_prolong<P>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, Phi, Ns, v, psi,
                           nrhs);
}
void launch_restrict64(const Geom& g, const c64* Phi, int Ns, const c64* psi, c64* w, int nrhs, hipStream_t s)
{
    restrict_any(g, Phi, Ns, psi, w, nrhs, s);
}
void launch_prolong64(const Geom& g, const c64* Phi, int Ns, const c64* v, c64* psi, int nrhs, hipStream_t s)
{
    prolong_any(g, Phi, Ns, v, psi, nrhs, s);
}
void launch_restrict_b32(const Geom& g, const c32* Phi, int Ns, const c64* psi, c64* w, int nrhs, hipStream_t s)
{
    restrict_any(g, Phi, Ns, psi, w, nrhs, s);
}
void launch_prolong_b32(const Geom& g, const c32* Phi, int Ns, const c64* v, c64* psi, int nrhs, hipStream_t s)
{
    prolong_any(g, Phi, Ns, v, psi, nrhs, s);
}
bool launch_block_gs64(const Geom& g, c64* F, int Ns, double rank_tol, int* flag, c64* R, hipStream_t s, c64* FT,
                       c32* F32)
{
    const int e = (12 * (int)g.Vb + kBT - 1) / kBT;  // entries per thread
    if (e <= 6)
        hipLaunchKernelGGL(k_block_gs<6>, dim3(g.Nb), dim3(kBT), 0, s, g, F, Ns, rank_tol, flag, R);
    else if (e <= 12 && g.Vb % kTile == 0) {  // kGsGroup fields at a time, 512 threads: six entries of each per thread
        hipLaunchKernelGGL((k_block_gsg<6, 512, kGsGroup>), dim3(g.Nb), dim3(512), 0, s, g, F, Ns, rank_tol, flag, R,
                           FT, F32);
        return true;
    } else if (e <= 12)
        hipLaunchKernelGGL((k_block_gsg<6, 512, kGsGroup>), dim3(g.Nb), dim3(512), 0, s, g, F, Ns, rank_tol, flag, R,
                           nullptr, nullptr);
    else if (e <= 24)
        hipLaunchKernelGGL(k_block_gs<24>, dim3(g.Nb), dim3(kBT), 0, s, g, F, Ns, rank_tol, flag, R);
    else
        hipLaunchKernelGGL(k_block_gs_stream, dim3(g.Nb), dim3(kBT), 0, s, g, F, Ns, rank_tol, flag, R);
    return FT == nullptr && F32 == nullptr;
}
int little_columns_max(int Ns)
{
    int nc = kMaxPairs * 256 / Ns;
    return nc < 1 ? 1 : nc;
}

bool little_columns_transposable(int Ns, int nc) { return Ns <= 24 && nc <= 4 * kRtJ; }

void launch_little_columns64(const Geom& g, const c64* Phi, int Ns, const c64* Y, int nc, int l0, int d, c64* A,
                             c64* part, long part_cap, hipStream_t s, bool transposed)
{
    if (transposed && (d == 0 || !little_columns_transposable(Ns, nc)))
        fail(DFL_EINVAL, "little-operator assembly: transposed order only for face columns of the tiled kernels");
    const size_t lds = sizeof(c64) * (Ns + nc) * (kCE + 1);
    // columns of a block hop: only the face towards the neighbour (see k_little_columns)
    const int fmu = d == 0 ? -1 : (d - 1) / 2;
    const int fy = d == 0 ? 0 : ((d & 1) ? g.b[fmu] - 1 : 0);
    const int nface = fmu < 0 ? g.Vb : g.Vb / g.b[fmu];
    const int ne = 12 * nface;
    int nsplit = ne / (8 * kCE);  // at least 8 staged tiles per workgroup
    if (nsplit > 8)
        nsplit = 8;
    while (nsplit > 1 && (long)nsplit * g.Nb * Ns * nc > part_cap)
        --nsplit;
    if (nsplit < 1)
        nsplit = 1;
    if ((long)nsplit * g.Nb * Ns * nc > part_cap)
        fail(DFL_EINVAL, "little-operator assembly: scratch too small for the column chunk");
    const size_t lds_rt = sizeof(c64) * (Ns + nc) * kRtCE;
    if (Ns <= 20 && nc <= 4 * kRtJ) {
        if (transposed)
            hipLaunchKernelGGL((k_little_columns_rt<5, true>), dim3(g.Nb * nsplit), dim3(256), lds_rt, s, g, Phi, Ns, Y,
                               nc, nsplit, fmu, fy, nface, part);
        else
            hipLaunchKernelGGL((k_little_columns_rt<5, false>), dim3(g.Nb * nsplit), dim3(256), lds_rt, s, g, Phi, Ns,
                               Y, nc, nsplit, fmu, fy, nface, part);
    } else if (Ns <= 24 && nc <= 4 * kRtJ) {
        if (transposed)
            hipLaunchKernelGGL((k_little_columns_rt<6, true>), dim3(g.Nb * nsplit), dim3(256), lds_rt, s, g, Phi, Ns, Y,
                               nc, nsplit, fmu, fy, nface, part);
        else
            hipLaunchKernelGGL((k_little_columns_rt<6, false>), dim3(g.Nb * nsplit), dim3(256), lds_rt, s, g, Phi, Ns,
                               Y, nc, nsplit, fmu, fy, nface, part);
    } else {
        static std::once_flag attr;
        set_max_lds_once(attr, reinterpret_cast<const void*>(&k_little_columns),
                         (int)(sizeof(c64) * (64 + 64) * (kCE + 1)));
        hipLaunchKernelGGL(k_little_columns, dim3(g.Nb * nsplit), dim3(256), lds, s, g, Phi, Ns, Y, nc, nsplit, fmu,
                           fy, nface, part);
    }
    const long n = (long)g.Nb * Ns * nc;
    hipLaunchKernelGGL(k_little_columns_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, part, Ns, nc,
                       nsplit, l0, d, A);
}

bool little_columns_all_ok(int Ns, long part_cap, long Nb) { return Ns >= 1 && Ns <= 32 && part_cap >= Nb * Ns * Ns; }

// dynamic LDS of k_little_columns_mfma: the staged rows or the wavefronts' tiles
size_t columns_mfma_lds(int Ns, int RT, int CT)
{
    return std::max(sizeof(c64) * 2 * Ns * kMfRow, sizeof(double) * 4 * RT * CT * 4 * 64);
}

template <int RT, int CT, bool TL>
void launch_columns_mfma(const Geom& g, const c64* Phi, int Ns, const c64* Y1, int n1, const c64* Y2, int nsplit,
                         int fmu, int fy, int nface, c64* part, hipStream_t s)
{
    static std::once_flag attr;  // the limit for the largest Ns of this tile count
    set_max_lds_once(attr, reinterpret_cast<const void*>(&k_little_columns_mfma<RT, CT, TL>),
                     (int)columns_mfma_lds(8 * RT, RT, CT));
    hipLaunchKernelGGL((k_little_columns_mfma<RT, CT, TL>), dim3(g.Nb * nsplit), dim3(256),
                       columns_mfma_lds(Ns, RT, CT), s, g, Phi, Ns, Y1, n1, Y2, nsplit, fmu, fy, nface, part);
}

void launch_little_columns64_all(const Geom& g, const c64* Phi, int Ns, const c64* Y1, int n1, const c64* Y2, int d,
                                 c64* A, c64* part, long part_cap, hipStream_t s, bool transposed)
{
    if (!little_columns_all_ok(Ns, part_cap, g.Nb) || n1 < 0 || n1 > Ns || (n1 < Ns && !Y2))
        fail(DFL_EINVAL, "little-operator assembly: all-column products need Ns <= 32 and Nb Ns^2 scratch entries");
    if (transposed && d == 0)
        fail(DFL_EINVAL, "little-operator assembly: transposed order only for face columns");
    const int fmu = d == 0 ? -1 : (d - 1) / 2;
    const int fy = d == 0 ? 0 : ((d & 1) ? g.b[fmu] - 1 : 0);
    const int nface = fmu < 0 ? g.Vb : g.Vb / g.b[fmu];
    const int ne = 12 * nface;
    // the entries of a block split over workgroups only when the blocks alone
    // give fewer than about eight workgroups per CU (on 64x32^3 one workgroup
    // per block and direction was 2 ms per setup faster than three or five
    // splits), each split at least four staged tiles
    int nsplit = (kColsMinGrid + g.Nb - 1) / g.Nb;
    nsplit = std::min({nsplit, 8, std::max(1, ne / (4 * kMfCE))});
    while (nsplit > 1 && (long)nsplit * g.Nb * Ns * Ns > part_cap)
        --nsplit;
    const int RT = (Ns + 7) / 8;  // CT = (Ns + 15) / 16 follows from RT
#define COLS_MFMA(R, C)                                                                                          \
    (transposed ? launch_columns_mfma<R, C, true>(g, Phi, Ns, Y1, n1, Y2, nsplit, fmu, fy, nface, part, s)      \
                : launch_columns_mfma<R, C, false>(g, Phi, Ns, Y1, n1, Y2, nsplit, fmu, fy, nface, part, s))
    switch (RT) {
    case 1: COLS_MFMA(1, 1); break;
    case 2: COLS_MFMA(2, 1); break;
    case 3: COLS_MFMA(3, 2); break;
    default: COLS_MFMA(4, 2); break;
    }
#undef COLS_MFMA
    const long n = (long)g.Nb * Ns * Ns;
    hipLaunchKernelGGL(k_little_columns_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, part, Ns, Ns,
                       nsplit, 0, d, A);
}

template <typename T>
void launch_little_apply(const Geom& g, const cpx<T>* A, int Ns, const cpx<T>* v, cpx<T>* w, int nrhs, hipStream_t s)
{
    long rows = (long)g.Nb * Ns;
    hipLaunchKernelGGL(k_little_apply<T>, dim3((unsigned)((rows + 255) / 256), nrhs), dim3(256), 0, s, g, A, Ns, v,
                       w);
}
template void launch_little_apply<double>(const Geom&, const c64*, int, const c64*, c64*, int, hipStream_t);
template void launch_little_apply<float>(const Geom&, const c32*, int, const c32*, c32*, int, hipStream_t);

void launch_little_apply_mfma(const Geom& g, const c32* At, int Ns, const c32* v, c32* w, int nrhs, hipStream_t s)
{
    const size_t lds = sizeof(c32) * 9 * Ns * kMfmaRhs;
    static std::once_flag attr;
    if (lds > 65536)
        set_max_lds_once(attr, reinterpret_cast<const void*>(&k_little_apply_mfma), 9 * 64 * kMfmaRhs * sizeof(c32));
    hipLaunchKernelGGL(k_little_apply_mfma, dim3(g.Nb), dim3(256), lds, s, g, At, Ns, v, w, nrhs);
}

void launch_little_eo_prep(const Geom& g, const c64* A, int Ns, c64* Mt64, c32* Mt32, int* flag, hipStream_t s)
{
    const size_t lds = sizeof(c64) * (2 * (size_t)Ns * Ns + Ns);
    static std::once_flag attr;
    set_max_lds_once(attr, reinterpret_cast<const void*>(&k_little_eo_prep), (int)(sizeof(c64) * (2 * 64 * 64 + 64)));
    hipLaunchKernelGGL(k_little_eo_prep, dim3(g.Nb), dim3(256), lds, s, g, A, Ns, Mt64, Mt32, flag);
}

void launch_global_modes(const Geom& g, const c64* R, int Ns, c64* U, hipStream_t s)
{
    const long n = (long)g.Nb * Ns * Ns;
    hipLaunchKernelGGL(k_global_modes, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, R, Ns, U);
}
void launch_eo_hop(const Geom& g, const c64* Mt, int Ns, const c64* in, const c64* sv, c64* out, int nv, int parity,
                   double alpha, double beta, hipStream_t s)
{
    const long N = (long)g.Nb * Ns;
    hipLaunchKernelGGL(k_eo_hop, dim3((unsigned)((N + 255) / 256), nv), dim3(256), 0, s, g, Mt, Ns, in, sv, out,
                       parity, alpha, beta);
}
void launch_gram(const c64* X, long n, int nv, c64* G, hipStream_t s)
{
    hipLaunchKernelGGL(k_gram, dim3(nv * nv), dim3(256), 0, s, X, n, nv, G);
}
void launch_gram2(const c64* X, const c64* Y, long n, int nv, c64* G, hipStream_t s)
{
    hipLaunchKernelGGL(k_gram2, dim3(nv * nv), dim3(256), 0, s, X, Y, n, nv, G);
}
void launch_combine(const c64* X, long n, int nv, int m, const c64* C, c64* Y, hipStream_t s)
{
    if (m > 0)
        hipLaunchKernelGGL(k_combine, dim3((unsigned)((n + 255) / 256), m), dim3(256), 0, s, X, n, nv, m, C, Y);
}

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
