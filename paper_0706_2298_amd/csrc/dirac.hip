// The Wilson-Dirac stencil (the operator of eq. (3.9)) on native fields.
//
// One thread per site, 256 sites per workgroup, one grid row per right-hand
// side (k_dirac_blk below stages a 256-site block's spinors in LDS). Per site the kernel reads the eight neighbour spinors, the four
// forward links and the four backward links U_mu(x - mu) (owned by the
// neighbour; they come from L2/MALL, not HBM), and writes one spinor. The
// workgroup numbering is XCD-aware (common.h): each XCD sweeps a contiguous
// range of sites so that neighbour reuse stays inside one L2.
#include <complex>
#include <type_traits>

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
        if (crosses_time(g, n, y, mu, step))
            negate(p);
        if (step > 0)
            hop_fwd_rt(mu, load_link(U, mu, s), p, acc);
        else
            hop_bwd_rt(mu, load_link(U, mu, t), p, acc);
    }
}

// Workgroup id -> (site chunk, right-hand side): XCD k sweeps its contiguous
// range of chunks, and for each chunk all right-hand sides back to back, so
// the chunk's links are read from HBM once and from L2 for the other RHS.
template <int MODE, typename T, typename L, bool CLV>
__global__ __launch_bounds__(256) void k_dirac(Geom g, L U, const cpx<T>* __restrict__ psi,
                                               cpx<T>* __restrict__ out, T diag, int hop_mu, int hop_dir,
                                               int chunks_padded, int nrhs, const cpx<T>* __restrict__ sub,
                                               Clover<T> C)
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
        const spinor<T> self = load_spinor(f, g.V, s);
        o = finish(self, acc, diag);
        if constexpr (CLV)
            clover_add(C, s, self, o);
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
template <typename T, typename L, bool CLV>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 4 : 2) void k_dirac_blk(Geom g, L U, const cpx<T>* __restrict__ psi,
                                                   cpx<T>* __restrict__ out, T diag, int chunks_padded, int nrhs,
                                                   const cpx<T>* __restrict__ sub, Clover<T> C)
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
    // x3 and x2 hops first: their neighbours across the block faces are
    // scattered partial lines of the neighbouring blocks, which run at the
    // same time on the same XCD and have just fetched those lines
#pragma unroll 1
    for (int h = 0; h < 8; ++h) {
        const int mu = 3 - (h >> 1);
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
            if (crosses_time(g, n, y, mu, step))
                negate(p);
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
    if constexpr (CLV)
        clover_add(C, s, self, o);
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

// ------------------------------------------------- 4^4 layout blocks
//
// Faces of a 4^4 block: face f = 2 (3 - mu) + (dir < 0), i.e. f = 0, 1 the
// forward and backward faces normal to x3, ..., f = 6, 7 those normal to x0.
// Each holds 64 sites, numbered by the other three in-block coordinates
// (ascending directions, the highest fastest). The kernels below load the
// neighbour spinors across the first NF faces in the same burst as the block's
// own spinors, spin-project them ((1 - g_mu) psi across a forward face,
// (1 + g_mu) psi across a backward one) and keep the two colour vectors in
// LDS, where the face sites' hops read them. In the native site order the
// neighbours across the x3 and x2 faces are every fourth site or runs of four
// sites of the neighbouring block, i.e. parts of its cache lines; that block
// runs at the same time on the same XCD, so a fetch in the same burst as its
// own loads is mostly an L2 hit instead of a second fetch later on.

constexpr int kFaceSites = 64;

__device__ inline int face_pos(const int y[4], int mu)
{
    int r = 0;
#pragma unroll
    for (int nu = 0; nu < 4; ++nu)
        if (nu != mu)
            r = r * 4 + y[nu];
    return r;
}

// thread t0 loads the neighbour across face (t0 / 64) + 4 k at face position
// t0 % 64, for k < NF / 4
template <int NF, typename T>
__device__ inline void face_load(const Geom& g, const cpx<T>* __restrict__ f, const int n[4], int t0,
                                 spinor<T> (&hp)[NF / 4])
{
#pragma unroll
    for (int k = 0; k < NF / 4; ++k) {
        const int fi = (t0 >> 6) + 4 * k;
        const int mu = 3 - (fi >> 1);
        const int step = (fi & 1) ? -1 : +1;
        int yy[4], nn[4];
        int rr = t0 & (kFaceSites - 1);
#pragma unroll
        for (int nu = 3; nu >= 0; --nu) {
            nn[nu] = n[nu];
            if (nu != mu) {
                yy[nu] = rr & 3;
                rr >>= 2;
            }
        }
        yy[mu] = step > 0 ? 0 : 3;
        nn[mu] = n[mu] + step;
        nn[mu] += nn[mu] < 0 ? g.nb[mu] : (nn[mu] >= g.nb[mu] ? -g.nb[mu] : 0);
        hp[k] = load_spinor(f, g.V, site_compose(g, nn, yy));
    }
}

// projects the loaded neighbours (with the antiperiodic sign of a hop across
// x0 = L0 - 1 <-> 0) into the face arrays
template <int NF, typename T>
__device__ inline void face_store(const Geom& g, const int n[4], int t0, spinor<T> (&hp)[NF / 4],
                                  cpx<T> (*hal)[6][kFaceSites])
{
#pragma unroll
    for (int k = 0; k < NF / 4; ++k) {
        const int fi = (t0 >> 6) + 4 * k;
        const int mu = 3 - (fi >> 1);
        const int step = (fi & 1) ? -1 : +1;
        if (mu == 0 && g.tsign < 0 && (step > 0 ? n[0] == g.nb[0] - 1 : n[0] == 0))
            negate(hp[k]);
        cvec3<T> a, b;
        proj_rt(mu, step, hp[k], a, b);
        const int r = t0 & (kFaceSites - 1);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            hal[fi][q][r] = a.c[q];
            hal[fi][3 + q][r] = b.c[q];
        }
    }
}

// hop H (order x3+, x3-, x2+, ..., x0-) of site s: the neighbour from the
// block's spinors in LDS, from the face arrays, or (faces >= NF) from memory
template <int H, int NF, typename T, typename L>
__device__ inline void hop4(const Geom& g, const cpx<T>* __restrict__ f, const cpx<T> (*sp)[256],
                            const cpx<T> (*hal)[6][kFaceSites], const LinkRows<L>& u, int t0, long s, const int n[4],
                            const int y[4], spinor<T>& acc)
{
    constexpr int MU = 3 - (H >> 1);
    constexpr int STEP = (H & 1) ? -1 : +1;
    constexpr int FI = H;
    constexpr int LSTR = MU == 3 ? 1 : MU == 2 ? 4 : MU == 1 ? 16 : 64;
    const bool inside = STEP > 0 ? y[MU] < 3 : y[MU] > 0;
    cvec3<T> a, b;
    if (inside) {
        spinor<T> p;
#pragma unroll
        for (int al = 0; al < 4; ++al)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                p.s[al].c[c] = sp[3 * al + c][t0 + STEP * LSTR];
        if (STEP > 0)
            proj_fwd<MU>(p, a, b);
        else
            proj_bwd<MU>(p, a, b);
    } else if (FI < NF) {
        const int r = face_pos(y, MU);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            a.c[q] = hal[FI][q][r];
            b.c[q] = hal[FI][3 + q][r];
        }
    } else {
        spinor<T> p = load_spinor(f, g.V, site_step(g, s, n, y, MU, STEP));
        if (crosses_time(g, n, y, MU, STEP))
            negate(p);
        if (STEP > 0)
            proj_fwd<MU>(p, a, b);
        else
            proj_bwd<MU>(p, a, b);
    }
    hop_add<MU, STEP>(to_link(u), a, b, acc);
}

// out (+ off) = diag psi - 1/2 acc (+ clover) at site s, or sub - that;
// non-temporal stores (the result is not re-read by this kernel)
template <typename T, bool CLV>
__device__ inline void finish_store(const cpx<T> (*sp)[256], int t0, long s, const spinor<T>& acc, T diag,
                                    const Clover<T>& C, const cpx<T>* __restrict__ sub, cpx<T>* __restrict__ dst)
{
    spinor<T> self;
#pragma unroll
    for (int al = 0; al < 4; ++al)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            self.s[al].c[a] = sp[3 * al + a][t0];
    spinor<T> o = finish(self, acc, diag);
    if constexpr (CLV)
        clover_add(C, s, self, o);
    if (sub) {
        const spinor<T> a = load_spinor(sub, 0, s);
#pragma unroll
        for (int al = 0; al < 4; ++al)
            o.s[al] = a.s[al] - o.s[al];
    }
#pragma unroll
    for (int al = 0; al < 4; ++al)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cpx<T>* q = reinterpret_cast<cpx<T>*>(reinterpret_cast<char*>(dst) + toff<cpx<T>>(s, 3 * al + a, 12));
            __builtin_nontemporal_store(o.s[al].c[a].re, &q->re);
            __builtin_nontemporal_store(o.s[al].c[a].im, &q->im);
        }
}

// FP32 spinors with FP32 links: one workgroup per (4^4 block, field); own
// spinors and all eight faces staged at the start, together with all eight
// links of every site (two rows each). Consecutive workgroups take the same
// block for the different fields, so that after the first field the links
// come from L2.
template <typename T, typename L, bool CLV>
__global__ __launch_bounds__(256, 2) void k_dirac_f4(Geom g, L U, const cpx<T>* __restrict__ psi,
                                                     cpx<T>* __restrict__ out, T diag, int chunks_padded, int nrhs,
                                                     const cpx<T>* __restrict__ sub, Clover<T> C)
{
    __shared__ cpx<T> sp[12][256];
    __shared__ cpx<T> hal[8][6][kFaceSites];
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
    int n[4], y[4];
    site_decompose(g, s, n, y);
    const spinor<T> own = load_spinor(f, g.V, s);
    spinor<T> hp[2];
    face_load<8>(g, f, n, t0, hp);
    LinkRows<L> uf[4], ub[4];
#pragma unroll
    for (int mu = 3; mu >= 0; --mu) {
        uf[mu] = load_rows(U, mu, s);
        ub[mu] = load_rows(U, mu, site_step(g, s, n, y, mu, -1));
    }
#pragma unroll
    for (int c = 0; c < 12; ++c)
        sp[c][t0] = own.s[c / 3].c[c % 3];
    face_store<8>(g, n, t0, hp, hal);
    __syncthreads();
    spinor<T> acc;
    zero(acc);
    hop4<0, 8>(g, f, sp, hal, uf[3], t0, s, n, y, acc);
    hop4<1, 8>(g, f, sp, hal, ub[3], t0, s, n, y, acc);
    hop4<2, 8>(g, f, sp, hal, uf[2], t0, s, n, y, acc);
    hop4<3, 8>(g, f, sp, hal, ub[2], t0, s, n, y, acc);
    hop4<4, 8>(g, f, sp, hal, uf[1], t0, s, n, y, acc);
    hop4<5, 8>(g, f, sp, hal, ub[1], t0, s, n, y, acc);
    hop4<6, 8>(g, f, sp, hal, uf[0], t0, s, n, y, acc);
    hop4<7, 8>(g, f, sp, hal, ub[0], t0, s, n, y, acc);
    finish_store<T, CLV>(sp, t0, s, acc, diag, C, sub ? sub + off : nullptr, out + off);
}

// As k_dirac_f4 for BF16 links: the hop loop kept rolled and each hop's link
// loaded one hop ahead (three workgroups per CU).
template <typename T, typename L, bool CLV>
__global__ __launch_bounds__(256, 3) void k_dirac_f4p(Geom g, L U, const cpx<T>* __restrict__ psi,
                                                      cpx<T>* __restrict__ out, T diag, int chunks_padded, int nrhs,
                                                      const cpx<T>* __restrict__ sub, Clover<T> C)
{
    __shared__ cpx<T> sp[12][256];
    __shared__ cpx<T> hal[8][6][kFaceSites];
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
    int n[4], y[4];
    site_decompose(g, s, n, y);
    const spinor<T> own = load_spinor(f, g.V, s);
    spinor<T> hp[2];
    face_load<8>(g, f, n, t0, hp);
#pragma unroll
    for (int c = 0; c < 12; ++c)
        sp[c][t0] = own.s[c / 3].c[c % 3];
    face_store<8>(g, n, t0, hp, hal);
    __syncthreads();
    spinor<T> acc;
    zero(acc);
    LinkRows<L> next = load_rows(U, 3, s);
#pragma unroll 1
    for (int h = 0; h < 8; ++h) {
        const int mu = 3 - (h >> 1);
        const int step = (h & 1) ? -1 : +1;
        const LinkRows<L> cur = next;
        if (h < 7) {
            const int mu2 = 3 - ((h + 1) >> 1);
            next = load_rows(U, mu2, ((h + 1) & 1) ? site_step(g, s, n, y, mu2, -1) : s);
        }
        const bool inside = step > 0 ? y[mu] < 3 : y[mu] > 0;
        cvec3<T> a, b;
        if (inside) {
            spinor<T> p;
            const int tl = t0 + step * g.lstr[mu];
#pragma unroll
            for (int al = 0; al < 4; ++al)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    p.s[al].c[c] = sp[3 * al + c][tl];
            proj_rt(mu, step, p, a, b);
        } else {
            const int r = face_pos(y, mu);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                a.c[q] = hal[h][q][r];
                b.c[q] = hal[h][3 + q][r];
            }
        }
        hop_add_rt(mu, step, to_link(cur), a, b, acc);
    }
    finish_store<T, CLV>(sp, t0, s, acc, diag, C, sub ? sub + off : nullptr, out + off);
}

// The block-crossing hop (hop_mu, hop_dir) of MODE 2 on the sites it reaches
// only: one thread per site of the face {y_mu = b_mu - 1} (dir = +1) or
// {y_mu = 0} (dir = -1) of every layout block, for the nrhs fields in turn
// (the link is loaded once and serves them all). The other sites of out are
// left untouched (the little-operator assembly reads the face only). TL: psi
// and out in the transposed in-block order (site_compose_t), the face sites
// enumerated in that order (links always in the native one).
template <typename T, typename L, bool TL>
__global__ __launch_bounds__(256) void k_dirac_face(Geom g, L U, const cpx<T>* __restrict__ psi,
                                                    cpx<T>* __restrict__ out, int mu, int dir, int nface, int nrhs)
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
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int nu = TL ? q : 3 - q;  // fastest in-block coordinate first
        if (nu == mu) {
            y[nu] = dir > 0 ? g.b[nu] - 1 : 0;
        } else {
            y[nu] = r % g.b[nu];
            r /= g.b[nu];
        }
    }
    const long s = site_compose(g, n, y);
    const long so = TL ? site_compose_t(g, n, y) : s;
    const long fs = 12 * g.V;  // field stride
    spinor<T> z;
    zero(z);
    if (g.nb[mu] <= 1) {
        for (int q = 0; q < nrhs; ++q)
            store_spinor(out + q * fs, g.V, so, z);
        return;
    }
    const long t = site_step(g, s, n, y, mu, dir);
    long ti = t;
    if (TL) {
        int nn[4] = {n[0], n[1], n[2], n[3]}, yn[4] = {y[0], y[1], y[2], y[3]};
        yn[mu] = dir > 0 ? 0 : g.b[mu] - 1;  // the face hop always leaves the block
        nn[mu] = (n[mu] + dir + g.nb[mu]) % g.nb[mu];
        ti = site_compose_t(g, nn, yn);
    }
    const bool neg = crosses_time(g, n, y, mu, dir);
    const su3<T> u = load_link(U, mu, dir > 0 ? s : t);
    for (int q = 0; q < nrhs; ++q) {
        spinor<T> p0 = load_spinor(psi + q * fs, g.V, ti);
        if (neg)
            negate(p0);
        spinor<T> a0;
        zero(a0);
        if (dir > 0)
            hop_fwd_rt(mu, u, p0, a0);
        else
            hop_bwd_rt(mu, u, p0, a0);
        store_spinor(out + q * fs, g.V, so, finish(z, a0, T(0)));
    }
}

// dst = src with every block's sites in the transposed in-block order, for
// nf fields; one thread per (site, field)
__global__ __launch_bounds__(256) void k_to_transposed(Geom g, const c64* __restrict__ src, c64* __restrict__ dst)
{
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V)
        return;
    const long off = (long)blockIdx.y * 12 * g.V;
    int n[4], y[4];
    site_decompose(g, s, n, y);
    store_spinor(dst + off, g.V, site_compose_t(g, n, y), load_spinor(src + off, g.V, s));
}

// sub (MODE 0, may be null): out = sub - D psi; clov (may be null): the
// clover term, added in modes 0 and 1
template <typename X> struct same {
    using type = X;
};
template <int MODE, typename T, typename L>
void launch(const Geom& g, L U, const cpx<T>* psi, cpx<T>* out, int nrhs, T m0, int mu, int dir, hipStream_t s,
            const typename same<cpx<T>>::type* sub, const typename same<cpx<T>>::type* clov)
{
    const Clover<T> C{MODE == 2 ? nullptr : clov};
    const bool b4 = g.b[0] == 4 && g.b[1] == 4 && g.b[2] == 4 && g.b[3] == 4;
    if constexpr (MODE == 0 && sizeof(T) == 4) {
        if (b4) {
            const int gp = pad_grid(g.Nb);
            if constexpr (std::is_same<L, LinksBF16>::value) {
                if (C.c)
                    hipLaunchKernelGGL((k_dirac_f4p<T, L, true>), dim3(gp * nrhs), dim3(256), 0, s, g, U, psi,
                                       out, T(4) + m0, gp, nrhs, sub, C);
                else
                    hipLaunchKernelGGL((k_dirac_f4p<T, L, false>), dim3(gp * nrhs), dim3(256), 0, s, g, U, psi,
                                       out, T(4) + m0, gp, nrhs, sub, C);
            } else {
                if (C.c)
                    hipLaunchKernelGGL((k_dirac_f4<T, L, true>), dim3(gp * nrhs), dim3(256), 0, s, g, U, psi,
                                       out, T(4) + m0, gp, nrhs, sub, C);
                else
                    hipLaunchKernelGGL((k_dirac_f4<T, L, false>), dim3(gp * nrhs), dim3(256), 0, s, g, U, psi,
                                       out, T(4) + m0, gp, nrhs, sub, C);
            }
            return;
        }
    }
    if (MODE == 0 && g.Vb == 256) {
        const int gp = pad_grid(g.Nb);
        if (C.c)
            hipLaunchKernelGGL((k_dirac_blk<T, L, true>), dim3(gp * nrhs), dim3(256), 0, s, g, U, psi, out,
                               T(4) + m0, gp, nrhs, sub, C);
        else
            hipLaunchKernelGGL((k_dirac_blk<T, L, false>), dim3(gp * nrhs), dim3(256), 0, s, g, U, psi, out,
                               T(4) + m0, gp, nrhs, sub, C);
        return;
    }
    long nwg = (g.V + 255) / 256;
    int gp = pad_grid(nwg);
    if (MODE != 2 && C.c)
        hipLaunchKernelGGL((k_dirac<MODE, T, L, true>), dim3(gp * nrhs), dim3(256), 0, s, g, U, psi, out, T(4) + m0,
                           mu, dir, gp, nrhs, MODE == 0 ? sub : nullptr, C);
    else
        hipLaunchKernelGGL((k_dirac<MODE, T, L, false>), dim3(gp * nrhs), dim3(256), 0, s, g, U, psi, out,
                           T(4) + m0, mu, dir, gp, nrhs, MODE == 0 ? sub : nullptr, C);
}

}  // namespace

void launch_dirac64(const Geom& g, Links64 U, const c64* psi, c64* out, int nrhs, double m0, int mode, int mu,
                    int dir, hipStream_t s, const c64* clov)
{
    if (mode == 0)
        launch<0>(g, U, psi, out, nrhs, m0, mu, dir, s, nullptr, clov);
    else if (mode == 1)
        launch<1>(g, U, psi, out, nrhs, m0, mu, dir, s, nullptr, clov);
    else
        launch<2>(g, U, psi, out, nrhs, m0, mu, dir, s, nullptr, nullptr);
}

void launch_dirac64_sub(const Geom& g, Links64 U, const c64* sub, const c64* psi, c64* out, int nrhs, double m0,
                        hipStream_t s, const c64* clov)
{
    launch<0>(g, U, psi, out, nrhs, m0, 0, 0, s, sub, clov);
}

void launch_dirac64_face(const Geom& g, Links64 U, const c64* psi, c64* out, int nrhs, int mu, int dir, hipStream_t s,
                         bool transposed)
{
    const int nface = (int)(g.Vb / g.b[mu]);
    const long n = (long)g.Nb * nface;
    if (transposed)
        hipLaunchKernelGGL((k_dirac_face<double, Links64, true>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           g, U, psi, out, mu, dir, nface, nrhs);
    else
        hipLaunchKernelGGL((k_dirac_face<double, Links64, false>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           g, U, psi, out, mu, dir, nface, nrhs);
}

void launch_to_transposed(const Geom& g, const c64* src, c64* dst, int nf, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_transposed, dim3((unsigned)((g.V + 255) / 256), nf), dim3(256), 0, s, g, src, dst);
}

void launch_dirac32(const Geom& g, Links32 U, const c32* psi, c32* out, int nrhs, float m0, hipStream_t s,
                    const c32* clov)
{
    launch<0>(g, U, psi, out, nrhs, m0, 0, 0, s, nullptr, clov);
}

void launch_dirac_bf16(const Geom& g, LinksBF16 U, const c32* psi, c32* out, int nrhs, float m0, hipStream_t s,
                       const c32* clov)
{
    launch<0>(g, U, psi, out, nrhs, m0, 0, 0, s, nullptr, clov);
}

}  // namespace dfl

// ------------------------------------------------------------ clover term

namespace dfl {

namespace {

// sigma_{mu nu} restricted to one chirality (2 x 2), for the six planes mu < nu
struct SigmaBlocks {
    c64 s[6][2][2][2];  // [plane][chirality][row][col]
};

__device__ inline su3<double> mat_mul(const su3<double>& a, const su3<double>& b)
{
    su3<double> c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            c.m[i][j] = a.m[i][0] * b.m[0][j] + a.m[i][1] * b.m[1][j] + a.m[i][2] * b.m[2][j];
    return c;
}

__device__ inline su3<double> dag(const su3<double>& a)
{
    su3<double> c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            c.m[i][j] = conjg(a.m[j][i]);
    return c;
}

// native index of the site x + step * mu
__device__ inline long shifted(const Geom& g, long s, int mu, int step)
{
    int n[4], y[4];
    site_decompose(g, s, n, y);
    return site_step(g, s, n, y, mu, step);
}

// Fhat_{mu nu}(x) = (Q - Q^+) / 8, Q = sum of the four plaquette leaves in
// the (mu, nu) plane that start and end at x (counter-clockwise from the
// mu direction)
__device__ inline su3<double> field_tensor(const Geom& g, const Links64& U, long x, int mu, int nu)
{
    const long xpm = shifted(g, x, mu, +1), xpn = shifted(g, x, nu, +1);
    const long xmm = shifted(g, x, mu, -1), xmn = shifted(g, x, nu, -1);
    const long xmm_pn = shifted(g, xmm, nu, +1), xmm_mn = shifted(g, xmm, nu, -1);
    const long xmn_pm = shifted(g, xmn, mu, +1);
    su3<double> Q = mat_mul(mat_mul(load_link(U, mu, x), load_link(U, nu, xpm)),
                            mat_mul(dag(load_link(U, mu, xpn)), dag(load_link(U, nu, x))));
    su3<double> l = mat_mul(mat_mul(load_link(U, nu, x), dag(load_link(U, mu, xmm_pn))),
                            mat_mul(dag(load_link(U, nu, xmm)), load_link(U, mu, xmm)));
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Q.m[i][j] += l.m[i][j];
    l = mat_mul(mat_mul(dag(load_link(U, mu, xmm)), dag(load_link(U, nu, xmm_mn))),
                mat_mul(load_link(U, mu, xmm_mn), load_link(U, nu, xmn)));
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Q.m[i][j] += l.m[i][j];
    l = mat_mul(mat_mul(dag(load_link(U, nu, xmn)), load_link(U, mu, xmn)),
                mat_mul(load_link(U, nu, xmn_pm), dag(load_link(U, mu, x))));
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Q.m[i][j] += l.m[i][j];
    su3<double> F;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const c64 a = Q.m[i][j], b = conjg(Q.m[j][i]);
            F.m[i][j] = c64{0.125 * (a.re - b.re), 0.125 * (a.im - b.im)};
        }
    return F;
}

// One thread per site: C_h = csw (i/2) sum_{mu < nu} sigma^h_{mu nu} (x) Fhat_{mu nu}
// for both chiralities h, written in the packed hermitian form of hop.h.
__global__ __launch_bounds__(256) void k_clover_field(Geom g, Links64 U, double csw, SigmaBlocks sig,
                                                      c64* __restrict__ C64, c32* __restrict__ C32)
{
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V)
        return;
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
        // one chirality at a time (Fhat is recomputed for the second): the
        // 6 x 6 block stays in registers
        c64 C[6][6];
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = 0; j < 6; ++j)
                C[i][j] = c64{0.0, 0.0};
        int plane = 0;
#pragma unroll 1
        for (int mu = 0; mu < 4; ++mu)
#pragma unroll 1
            for (int nu = mu + 1; nu < 4; ++nu, ++plane) {
                const su3<double> F = field_tensor(g, U, s, mu, nu);
#pragma unroll
                for (int al = 0; al < 2; ++al)
#pragma unroll
                    for (int be = 0; be < 2; ++be) {
                        // csw (i/2) sigma_{al be}
                        const c64 sg = sig.s[plane][h][al][be];
                        const c64 f = c64{-0.5 * csw * sg.im, 0.5 * csw * sg.re};
#pragma unroll
                        for (int a = 0; a < 3; ++a)
#pragma unroll
                            for (int b = 0; b < 3; ++b)
                                C[3 * al + a][3 * be + b] += f * F.m[a][b];
                    }
            }
        c64 e[18];
#pragma unroll
        for (int q = 0; q < 3; ++q)
            e[q] = c64{C[2 * q][2 * q].re, C[2 * q + 1][2 * q + 1].re};
        int q = 3;
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = i + 1; j < 6; ++j, ++q)
                e[q] = C[i][j];
#pragma unroll
        for (int q2 = 0; q2 < 18; ++q2) {
            st(C64, toff<c64>(s, 18 * h + q2, kCloverComp), e[q2]);
            if (C32)
                st(C32, toff<c32>(s, 18 * h + q2, kCloverComp), c32{(float)e[q2].re, (float)e[q2].im});
        }
    }
}

}  // namespace

void launch_clover_field(const Geom& g, Links64 U, double csw, c64* C64, c32* C32, hipStream_t s)
{
    // sigma_{mu nu} = (i/2) [g_mu, g_nu] is block diagonal in the chiral basis:
    // (i/2)(e_mu e_nu^+ - e_nu e_mu^+) on spins 0, 1 and
    // (i/2)(e_mu^+ e_nu - e_nu^+ e_mu) on spins 2, 3
    using cd = std::complex<double>;
    const cd I(0.0, 1.0);
    cd e[4][2][2] = {{{-1.0, 0.0}, {0.0, -1.0}},
                     {{0.0, -I}, {-I, 0.0}},
                     {{0.0, -1.0}, {1.0, 0.0}},
                     {{-I, 0.0}, {0.0, I}}};
    auto prod = [&](int a, bool da, int b, bool db, int i, int j) {
        cd t = 0.0;
        for (int k = 0; k < 2; ++k) {
            cd x = da ? std::conj(e[a][k][i]) : e[a][i][k];
            cd y = db ? std::conj(e[b][j][k]) : e[b][k][j];
            t += x * y;
        }
        return t;
    };
    SigmaBlocks sig;
    int plane = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu, ++plane)
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) {
                    cd up = 0.5 * I * (prod(mu, false, nu, true, i, j) - prod(nu, false, mu, true, i, j));
                    cd lo = 0.5 * I * (prod(mu, true, nu, false, i, j) - prod(nu, true, mu, false, i, j));
                    sig.s[plane][0][i][j] = c64{up.real(), up.imag()};
                    sig.s[plane][1][i][j] = c64{lo.real(), lo.imag()};
                }
    const unsigned nwg = (unsigned)((g.V + 255) / 256);
    hipLaunchKernelGGL(k_clover_field, dim3(nwg), dim3(256), 0, s, g, U, csw, sig, C64, C32);
}

}  // namespace dfl
