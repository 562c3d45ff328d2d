// The Wilson-Dirac stencil (the operator of eq. (3.9)) on native fields.
//
// One thread per site, 256 sites per workgroup, one grid row per right-hand
// side (k_dirac_blk below stages a 256-site block's spinors in LDS). Per site the kernel reads the eight neighbour spinors, the four
// forward links and the four backward links U_mu(x - mu) (owned by the
// neighbour; they come from L2/MALL, not HBM), and writes one spinor. The
// workgroup numbering is XCD-aware (common.h): each XCD sweeps a contiguous
// range of sites so that neighbour reuse stays inside one L2.
#include "hop.h"

namespace dfl {

namespace {

// MODE 0: full operator; 1: direct sum of the block operators (hops leaving a
// layout block dropped); 2: only the block-crossing hop (hop_mu, hop_dir),
// without the mass term. The direction loop is kept rolled so that each
// direction's loads stay in their own basic block: unrolled, the scheduler
// hoists all 180 loads of a site and the kernel spills.
template <int MODE, typename T, typename L>
__device__ inline void hops_all(const Geom& g, const L& U, const cpx<T>* __restrict__ f, long s, const int n[4],
                                const int y[4], int hop_mu, int hop_dir, spinor<T>& acc)
{
#pragma unroll 1
    for (int h = 0; h < 8; ++h) {
        const int mu = h >> 1;
        const int step = (h & 1) ? -1 : +1;
        bool keep = true;
        if (MODE == 1) {
            keep = (step > 0 ? y[mu] + 1 < g.b[mu] : y[mu] > 0) || g.nb[mu] == 1;
        } else if (MODE == 2) {
            keep = hop_mu == mu && hop_dir == step && (step > 0 ? y[mu] + 1 == g.b[mu] : y[mu] == 0) &&
                   g.nb[mu] > 1;
        }
        if (!keep)
            continue;
        long t = site_step(g, s, n, y, mu, step);
        spinor<T> p = load_spinor(f, g.V, t);
        if (step > 0)
            hop_fwd_rt(mu, load_link(U, mu, s), p, acc);
        else
            hop_bwd_rt(mu, load_link(U, mu, t), p, acc);
    }
}

// Workgroup id -> (site chunk, right-hand side): XCD k sweeps its contiguous
// range of chunks, and for each chunk all right-hand sides back to back, so
// the chunk's links are read from HBM once and from L2 for the other RHS.
template <int MODE, typename T, typename L>
__global__ __launch_bounds__(256) void k_dirac(Geom g, L U, const cpx<T>* __restrict__ psi,
                                               cpx<T>* __restrict__ out, T diag, int hop_mu, int hop_dir,
                                               int chunks_padded, int nrhs, const cpx<T>* __restrict__ sub)
{
    const int per = chunks_padded / kNumXcd;
    const int local = blockIdx.x / kNumXcd;
    const int wg = (blockIdx.x % kNumXcd) * per + local / nrhs;
    const int rhs = local % nrhs;
    long s = (long)wg * 256 + threadIdx.x;
    if (s >= g.V)
        return;
    long off = (long)rhs * 12 * g.V;
    const cpx<T>* f = psi + off;
    int n[4], y[4];
    site_decompose(g, s, n, y);
    spinor<T> acc;
    zero(acc);
    hops_all<MODE>(g, U, f, s, n, y, hop_mu, hop_dir, acc);
    spinor<T> o;
    if (MODE == 2) {
        spinor<T> z;
        zero(z);
        o = finish(z, acc, T(0));
    } else {
        o = finish(load_spinor(f, g.V, s), acc, diag);
    }
    if (sub) {
        const spinor<T> a = load_spinor(sub + off, g.V, s);
#pragma unroll
        for (int al = 0; al < 4; ++al)
            o.s[al] = a.s[al] - o.s[al];
    }
    store_spinor(out + off, g.V, s, o);
}

// Full operator for 256-site layout blocks with the block's spinors staged in
// LDS: one workgroup per (block, right-hand side), one thread per site; hops
// that stay inside the block read the neighbour from LDS (three quarters of
// them for 4^4 blocks), the others and all links come from global memory.
// The output is written with non-temporal stores (it is not re-read here).
template <typename T, typename L>
__global__ __launch_bounds__(256) void k_dirac_blk(Geom g, L U, const cpx<T>* __restrict__ psi,
                                                   cpx<T>* __restrict__ out, T diag, int chunks_padded, int nrhs,
                                                   const cpx<T>* __restrict__ sub)
{
    __shared__ cpx<T> sp[12][256];
    const int per = chunks_padded / kNumXcd;
    const int local = blockIdx.x / kNumXcd;
    const int blk = (blockIdx.x % kNumXcd) * per + local / nrhs;
    const int rhs = local % nrhs;
    if (blk >= g.Nb)
        return;
    const int t0 = threadIdx.x;
    const long s = (long)blk * 256 + t0;
    const long off = (long)rhs * 12 * g.V;
    const cpx<T>* f = psi + off;
#pragma unroll
    for (int c = 0; c < 12; ++c)
        sp[c][t0] = ld(f, toff<cpx<T>>(s, c, 12));
    __syncthreads();
    int n[4], y[4];
    site_decompose(g, s, n, y);
    spinor<T> acc;
    zero(acc);
#pragma unroll 1
    for (int h = 0; h < 8; ++h) {
        const int mu = h >> 1;
        const int step = (h & 1) ? -1 : +1;
        const bool inside = step > 0 ? y[mu] + 1 < g.b[mu] : y[mu] > 0;
        const long t = site_step(g, s, n, y, mu, step);
        spinor<T> p;
        if (inside) {
            const int tl = t0 + step * g.lstr[mu];
#pragma unroll
            for (int al = 0; al < 4; ++al)
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    p.s[al].c[a] = sp[3 * al + a][tl];
        } else {
            p = load_spinor(f, g.V, t);
        }
        if (step > 0)
            hop_fwd_rt(mu, load_link(U, mu, s), p, acc);
        else
            hop_bwd_rt(mu, load_link(U, mu, t), p, acc);
    }
    spinor<T> self;
#pragma unroll
    for (int al = 0; al < 4; ++al)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            self.s[al].c[a] = sp[3 * al + a][t0];
    spinor<T> o = finish(self, acc, diag);
    if (sub) {
        const spinor<T> a = load_spinor(sub + off, g.V, s);
#pragma unroll
        for (int al = 0; al < 4; ++al)
            o.s[al] = a.s[al] - o.s[al];
    }
    cpx<T>* dst = out + off;
#pragma unroll
    for (int al = 0; al < 4; ++al)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cpx<T>* q = reinterpret_cast<cpx<T>*>(reinterpret_cast<char*>(dst) + toff<cpx<T>>(s, 3 * al + a, 12));
            __builtin_nontemporal_store(o.s[al].c[a].re, &q->re);
            __builtin_nontemporal_store(o.s[al].c[a].im, &q->im);
        }
}

// The block-crossing hop (hop_mu, hop_dir) of MODE 2 on the sites it reaches
// only: one thread per site of the face {y_mu = b_mu - 1} (dir = +1) or
// {y_mu = 0} (dir = -1) of every layout block, blockIdx.y = right-hand side.
// The other sites of out are left untouched (the little-operator assembly
// reads the face only).
template <typename T, typename L>
__global__ __launch_bounds__(256) void k_dirac_face(Geom g, L U, const cpx<T>* __restrict__ psi,
                                                    cpx<T>* __restrict__ out, int mu, int dir, int nface)
{
    const long f = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= (long)g.Nb * nface)
        return;
    const int blk = (int)(f / nface);
    int r = (int)(f - (long)blk * nface), rb = blk;
    int n[4], y[4];
#pragma unroll
    for (int nu = 3; nu >= 0; --nu) {
        n[nu] = rb % g.nb[nu];
        rb /= g.nb[nu];
        if (nu == mu) {
            y[nu] = dir > 0 ? g.b[nu] - 1 : 0;
        } else {
            y[nu] = r % g.b[nu];
            r /= g.b[nu];
        }
    }
    const long s = site_compose(g, n, y);
    const long off = (long)blockIdx.y * 12 * g.V;
    spinor<T> acc;
    zero(acc);
    if (g.nb[mu] > 1) {
        const long t = site_step(g, s, n, y, mu, dir);
        spinor<T> p = load_spinor(psi + off, g.V, t);
        if (dir > 0)
            hop_fwd_rt(mu, load_link(U, mu, s), p, acc);
        else
            hop_bwd_rt(mu, load_link(U, mu, t), p, acc);
    }
    spinor<T> z;
    zero(z);
    store_spinor(out + off, g.V, s, finish(z, acc, T(0)));
}

// sub (MODE 0, may be null): out = sub - D psi
template <int MODE, typename T, typename L>
void launch(const Geom& g, L U, const cpx<T>* psi, cpx<T>* out, int nrhs, T m0, int mu, int dir, hipStream_t s,
            const cpx<T>* sub = nullptr)
{
    if (MODE == 0 && g.Vb == 256) {
        const int gp = pad_grid(g.Nb);
        hipLaunchKernelGGL((k_dirac_blk<T, L>), dim3(gp * nrhs), dim3(256), 0, s, g, U, psi, out, T(4) + m0, gp,
                           nrhs, sub);
        return;
    }
    long nwg = (g.V + 255) / 256;
    int gp = pad_grid(nwg);
    hipLaunchKernelGGL((k_dirac<MODE, T, L>), dim3(gp * nrhs), dim3(256), 0, s, g, U, psi, out, T(4) + m0, mu, dir,
                       gp, nrhs, MODE == 0 ? sub : nullptr);
}

}  // namespace

void launch_dirac64(const Geom& g, Links64 U, const c64* psi, c64* out, int nrhs, double m0, int mode, int mu,
                    int dir, hipStream_t s)
{
    if (mode == 0)
        launch<0>(g, U, psi, out, nrhs, m0, mu, dir, s);
    else if (mode == 1)
        launch<1>(g, U, psi, out, nrhs, m0, mu, dir, s);
    else
        launch<2>(g, U, psi, out, nrhs, m0, mu, dir, s);
}

void launch_dirac64_sub(const Geom& g, Links64 U, const c64* sub, const c64* psi, c64* out, int nrhs, double m0,
                        hipStream_t s)
{
    launch<0>(g, U, psi, out, nrhs, m0, 0, 0, s, sub);
}

void launch_dirac64_face(const Geom& g, Links64 U, const c64* psi, c64* out, int nrhs, int mu, int dir, hipStream_t s)
{
    const int nface = (int)(g.Vb / g.b[mu]);
    const long n = (long)g.Nb * nface;
    hipLaunchKernelGGL((k_dirac_face<double, Links64>), dim3((unsigned)((n + 255) / 256), nrhs), dim3(256), 0, s, g,
                       U, psi, out, mu, dir, nface);
}

void launch_dirac32(const Geom& g, Links32 U, const c32* psi, c32* out, int nrhs, float m0, hipStream_t s)
{
    launch<0>(g, U, psi, out, nrhs, m0, 0, 0, s);
}

void launch_dirac_bf16(const Geom& g, LinksBF16 U, const c32* psi, c32* out, int nrhs, float m0, hipStream_t s)
{
    launch<0>(g, U, psi, out, nrhs, m0, 0, 0, s);
}

}  // namespace dfl
