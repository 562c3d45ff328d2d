// One colour sweep of the Schwarz alternating procedure: every Schwarz block
// of the given colour computes its residual r = (rho - D psi)|_Lambda with the
// full operator, runs nmr minimal-residual steps on the block operator
// D_Lambda (Dirichlet walls) and adds the block solution to psi.
//
// Mapping: one workgroup per Schwarz block. The generic kernel (k_sap, any
// block size, FP64 or FP32) and the several-field kernel (k_sap_rl, blocks of
// at most 256 sites) run one thread per site (blockDim = |block| rounded up to
// a wavefront; spare lanes only join the reductions); the one-field kernel
// (k_sap_pair) runs two lanes per site. The residual reads the neighbour
// spinors across the block faces directly from global memory; those sites
// belong to blocks of the other colour, which no workgroup of this launch
// writes, so there is no race. Inside the MR loop the current residue r is
// exchanged through LDS (12 planes x |block|), and the two block reductions
// per step use DPP wavefront sums plus one LDS pass. k_sap reads the links
// through L1/L2 at every MR step; k_sap_rl and k_sap_pair keep them from the
// residual on.
//
// init (first cycle, where psi starts at zero): 2 = psi is zero everywhere
// (colour 0: the residue is rho, no hops, no reads of psi), 1 = psi is zero on
// the sweep's own blocks (colour 1: only the neighbours' values are read).
// out64 (optional, last cycle of an FP32 sweep): the block's new psi is also
// written in FP64 there, so no conversion pass follows.
#include "hop.h"

namespace dfl {

namespace {

// factor of field b's rho when it enters scaled: 1 / sqrt(nrm2[2 b]) (0 for
// a zero field), 1 without nrm2
template <typename T> __device__ inline T rho_scale(const double* nrm2, int b)
{
    if (!nrm2)
        return T(1);
    const double q = nrm2[2 * b];
    return q > 0.0 ? (T)(1.0 / sqrt(q)) : T(0);
}
template <typename T> __device__ inline void scale_spinor(spinor<T>& p, T f)
{
#pragma unroll
    for (int al = 0; al < 4; ++al)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            p.s[al].c[a] = cpx<T>{p.s[al].c[a].re * f, p.s[al].c[a].im * f};
}

template <typename T> __device__ inline void store_spinor_f64(c64* __restrict__ f, long V, long s, const spinor<T>& p)
{
    spinor<double> d;
#pragma unroll
    for (int al = 0; al < 4; ++al)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            d.s[al].c[a] = c64{(double)p.s[al].c[a].re, (double)p.s[al].c[a].im};
    store_spinor(f, V, s, d);
}

// D_Lambda hops of one site: neighbours inside the Schwarz block come from
// the LDS copy of the residue; hops leaving the block are dropped.
template <typename T, typename L>
__device__ inline void block_hops(const Geom& g, const SapGeom& sg, const L& U, const cpx<T>* lr, int t,
                                  const int yl[4], long s, const int n[4], const int y[4], spinor<T>& acc)
{
    const int V = sg.Vsb;
#pragma unroll 1
    for (int h = 0; h < 8; ++h) {
        const int mu = h >> 1;
        const int step = (h & 1) ? -1 : +1;
        if (step > 0 ? yl[mu] + 1 >= sg.sb[mu] : yl[mu] == 0)
            continue;
        const int tn = t + step * sg.lstr[mu];
        spinor<T> p;
#pragma unroll
        for (int al = 0; al < 4; ++al)
#pragma unroll
            for (int a = 0; a < 3; ++a)
                p.s[al].c[a] = lr[(3 * al + a) * V + tn];
        if (step > 0)
            hop_fwd_rt(mu, load_link(U, mu, s), p, acc);
        else
            hop_bwd_rt(mu, load_link(U, mu, site_step(g, s, n, y, mu, -1)), p, acc);
    }
}

// the eight hops of the full operator at one site, neighbours from global
// memory; with outside_only, only the hops that leave the Schwarz block (the
// block's own psi is zero in the first cycle's colour-1 sweep)
template <typename T, typename L>
__device__ inline void full_hops(const Geom& g, const SapGeom& sg, const L& U, const cpx<T>* __restrict__ psi, long s,
                                 const int n[4], const int y[4], const int yl[4], bool outside_only, spinor<T>& acc)
{
#pragma unroll 1
    for (int h = 0; h < 8; ++h) {
        const int mu = h >> 1;
        const int step = (h & 1) ? -1 : +1;
        if (outside_only && (step > 0 ? yl[mu] + 1 < sg.sb[mu] : yl[mu] > 0))
            continue;
        long tn = site_step(g, s, n, y, mu, step);
        spinor<T> p = load_spinor(psi, g.V, tn);
        if (crosses_time(g, n, y, mu, step))
            negate(p);
        if (step > 0)
            hop_fwd_rt(mu, load_link(U, mu, s), p, acc);
        else
            hop_bwd_rt(mu, load_link(U, mu, tn), p, acc);
    }
}

template <typename T, typename L, bool CLV>
__global__ __launch_bounds__(512) void k_sap(Geom g, SapGeom sg, L U, const cpx<T>* __restrict__ rho,
                                             const double* __restrict__ rho_nrm2, cpx<T>* __restrict__ psi, T diag,
                                             int nmr, int colour, int nrhs, int init, c64* __restrict__ out64,
                                             Clover<T> C)
{
    // workgroup -> (block of this colour, right-hand side), right-hand sides fastest
    const T rs = rho_scale<T>(rho_nrm2, blockIdx.x % nrhs);
    rho += (long)(blockIdx.x % nrhs) * 12 * g.V;
    psi += (long)(blockIdx.x % nrhs) * 12 * g.V;
    if (out64)
        out64 += (long)(blockIdx.x % nrhs) * 12 * g.V;
    extern __shared__ char smem_raw[];
    cpx<T>* lr = reinterpret_cast<cpx<T>*>(smem_raw);
    __shared__ double red[3][8];

    const int t = threadIdx.x;
    const bool active = t < sg.Vsb;
    const int lane = t & 63, wid = t >> 6, nw = blockDim.x >> 6;

    // k-th block of this colour -> block coordinates m
    int k = blockIdx.x / nrhs;
    int half = sg.nsb[3] / 2;
    int m[4];
    int j = k % half;
    int rest = k / half;
    m[2] = rest % sg.nsb[2];
    rest /= sg.nsb[2];
    m[1] = rest % sg.nsb[1];
    m[0] = rest / sg.nsb[1];
    m[3] = 2 * j + ((colour + m[0] + m[1] + m[2]) & 1);

    int yl[4] = {0, 0, 0, 0};
    int n[4] = {0, 0, 0, 0}, y[4] = {0, 0, 0, 0};
    long s = 0;
    if (active) {
        int tt = t;
        yl[3] = tt % sg.sb[3];
        tt /= sg.sb[3];
        yl[2] = tt % sg.sb[2];
        tt /= sg.sb[2];
        yl[1] = tt % sg.sb[1];
        yl[0] = tt / sg.sb[1];
        for (int mu = 0; mu < 4; ++mu) {
            int x = m[mu] * sg.sb[mu] + yl[mu];
            n[mu] = x / g.b[mu];
            y[mu] = x - n[mu] * g.b[mu];
        }
        s = site_compose(g, n, y);
    }

    // residual with the full operator
    spinor<T> r, xs;
    zero(r);
    zero(xs);
    if (active) {
        spinor<T> acc, self;
        zero(acc);
        zero(self);
        if (init < 2)
            full_hops(g, sg, U, psi, s, n, y, yl, init == 1, acc);
        if (init == 0)
            self = load_spinor(psi, g.V, s);
        spinor<T> d = finish(self, acc, diag);
        if constexpr (CLV)
            if (init == 0)
                clover_add(C, s, self, d);
        spinor<T> b = load_spinor(rho, g.V, s);
        if (rho_nrm2)
            scale_spinor(b, rs);
#pragma unroll
        for (int al = 0; al < 4; ++al)
            r.s[al] = b.s[al] - d.s[al];
    }

    for (int step = 0; step < nmr; ++step) {
        if (active) {
#pragma unroll
            for (int al = 0; al < 4; ++al)
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    lr[(3 * al + a) * sg.Vsb + t] = r.s[al].c[a];
        }
        __syncthreads();
        spinor<T> q;
        zero(q);
        double qr_re = 0.0, qr_im = 0.0, qq = 0.0;
        if (active) {
            spinor<T> acc;
            zero(acc);
            block_hops(g, sg, U, lr, t, yl, s, n, y, acc);
            q = finish(r, acc, diag);
            if constexpr (CLV)
                clover_add(C, s, r, q);
#pragma unroll
            for (int al = 0; al < 4; ++al)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    double qa = (double)q.s[al].c[a].re, qb = (double)q.s[al].c[a].im;
                    double ra = (double)r.s[al].c[a].re, rb = (double)r.s[al].c[a].im;
                    qr_re += qa * ra + qb * rb;
                    qr_im += qa * rb - qb * ra;
                    qq += qa * qa + qb * qb;
                }
        }
        qr_re = wave_sum(qr_re);
        qr_im = wave_sum(qr_im);
        qq = wave_sum(qq);
        if (lane == 0) {
            red[0][wid] = qr_re;
            red[1][wid] = qr_im;
            red[2][wid] = qq;
        }
        __syncthreads();
        double sre = 0.0, sim = 0.0, sqq = 0.0;
        for (int w = 0; w < nw; ++w) {
            sre += red[0][w];
            sim += red[1][w];
            sqq += red[2][w];
        }
        if (!(sqq > 0.0))
            break;  // zero residue on this block: uniform across the workgroup
        cpx<T> alpha{(T)(sre / sqq), (T)(sim / sqq)};
#pragma unroll
        for (int al = 0; al < 4; ++al)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                xs.s[al].c[a] += alpha * r.s[al].c[a];
                r.s[al].c[a] -= alpha * q.s[al].c[a];
            }
    }

    if (active) {
        spinor<T> p;
        zero(p);
        if (init == 0)
            p = load_spinor(psi, g.V, s);
#pragma unroll
        for (int al = 0; al < 4; ++al)
            p.s[al] += xs.s[al];
        store_spinor(psi, g.V, s, p);
        if (out64)
            store_spinor_f64(out64, g.V, s, p);
    }
}

// FP32 sweep for several fields with the site's eight links kept for the MR
// steps: the first two rows in registers (96 VGPRs), the third row, formed
// once during the residual, in LDS (24 planes x block). The MR steps then read
// only LDS, and two blocks of up to 256 sites share a CU (2 x 72 KB of LDS).
template <typename L> struct Link2 {
    c32 e[6];
};

template <typename L> __device__ inline Link2<L> load_link2(const L& U, int mu, long s);
template <> __device__ inline Link2<Links32> load_link2(const Links32& U, int mu, long s)
{
    Link2<Links32> r;
#pragma unroll
    for (int k = 0; k < 6; ++k)
        r.e[k] = ld(U.u, toff<c32>(s, mu * 6 + k, 24));
    return r;
}
template <> __device__ inline Link2<LinksBF16> load_link2(const LinksBF16& U, int mu, long s)
{
    Link2<LinksBF16> r;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        uint32_t w = ld(U.u, toff<uint32_t>(s, mu * 6 + k, 24));
        r.e[k] = c32{bf16_to_f(w & 0xffffu), bf16_to_f(w >> 16)};
    }
    return r;
}
template <typename L> __device__ inline su3<float> expand(const Link2<L>& l)
{
    su3<float> u;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            u.m[a][b] = l.e[a * 3 + b];
    complete_third_row(u);
    return u;
}

// the link from its two register rows and its third row in LDS (entry b at l3[b * stride])
template <typename L> __device__ inline su3<float> expand_lds(const Link2<L>& l, const c32* l3, int stride)
{
    su3<float> u;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            u.m[a][b] = l.e[a * 3 + b];
#pragma unroll
    for (int b = 0; b < 3; ++b)
        u.m[2][b] = l3[b * stride];
    return u;
}

// B4: 4^4 blocks, whose extents, in-block strides and LDS plane size are
// compile-time constants (every LDS access of a hop is then an immediate
// offset from the thread's own address).
template <typename L, bool B4>
__global__ __launch_bounds__(256, 2) void k_sap_rl(Geom g, SapGeom sg, L U, const c32* __restrict__ rho,
                                               const double* __restrict__ rho_nrm2, c32* __restrict__ psi,
                                               float diag, int nmr, int colour, int nrhs, int init,
                                               c64* __restrict__ out64)
{
    const int Vsb = B4 ? 256 : sg.Vsb;
    int sbl[4], lst[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        sbl[mu] = B4 ? 4 : sg.sb[mu];
        lst[mu] = B4 ? (64 >> (2 * mu)) : sg.lstr[mu];
    }
    // workgroup -> (block of this colour, right-hand side), right-hand sides fastest
    const float rs = rho_scale<float>(rho_nrm2, blockIdx.x % nrhs);
    rho += (long)(blockIdx.x % nrhs) * 12 * g.V;
    psi += (long)(blockIdx.x % nrhs) * 12 * g.V;
    if (out64)
        out64 += (long)(blockIdx.x % nrhs) * 12 * g.V;
    extern __shared__ char smem_raw[];
    c32* lr = reinterpret_cast<c32*>(smem_raw);
    c32* l3 = lr + 12 * Vsb;  // third link rows: entry (3 h + b) * Vsb + site
    __shared__ double red[3][8];

    const int t = threadIdx.x;
    const bool active = t < Vsb;
    const int lane = t & 63, wid = t >> 6, nw = blockDim.x >> 6;

    int k = blockIdx.x / nrhs;
    int half = sg.nsb[3] / 2;
    int m[4];
    int j = k % half;
    int rest = k / half;
    m[2] = rest % sg.nsb[2];
    rest /= sg.nsb[2];
    m[1] = rest % sg.nsb[1];
    m[0] = rest / sg.nsb[1];
    m[3] = 2 * j + ((colour + m[0] + m[1] + m[2]) & 1);

    int yl[4] = {0, 0, 0, 0};
    int n[4] = {0, 0, 0, 0}, y[4] = {0, 0, 0, 0};
    long s = 0;
    if (active) {
        int tt = t;
        yl[3] = tt % sbl[3];
        tt /= sbl[3];
        yl[2] = tt % sbl[2];
        tt /= sbl[2];
        yl[1] = tt % sbl[1];
        yl[0] = tt / sbl[1];
        for (int mu = 0; mu < 4; ++mu) {
            int x = m[mu] * sbl[mu] + yl[mu];
            n[mu] = x / g.b[mu];
            y[mu] = x - n[mu] * g.b[mu];
        }
        s = site_compose(g, n, y);
    }

    // residual with the full operator; the links are kept for the MR steps
    Link2<L> lk[8];
    spinor<float> r, xs;
    zero(r);
    zero(xs);
    if (active) {
        spinor<float> acc, self;
        zero(acc);
        zero(self);
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const int mu = h >> 1;
            const int step = (h & 1) ? -1 : +1;
            long tn = site_step(g, s, n, y, mu, step);
            lk[h] = load_link2(U, mu, step > 0 ? s : tn);
            const su3<float> u = expand(lk[h]);
#pragma unroll
            for (int b = 0; b < 3; ++b)
                l3[(3 * h + b) * Vsb + t] = u.m[2][b];
            const bool inside = step > 0 ? yl[mu] + 1 < sbl[mu] : yl[mu] > 0;
            if (init == 0 || (init == 1 && !inside)) {
                spinor<float> p = load_spinor(psi, g.V, tn);
                if (step > 0)
                    hop_fwd_rt(mu, u, p, acc);
                else
                    hop_bwd_rt(mu, u, p, acc);
            }
            if (h & 1)
                asm volatile("" ::: "memory");  // two hops' loads in flight at a time
        }
        if (init == 0)
            self = load_spinor(psi, g.V, s);
        spinor<float> d = finish(self, acc, diag);
        spinor<float> b = load_spinor(rho, g.V, s);
        if (rho_nrm2)
            scale_spinor(b, rs);
#pragma unroll
        for (int al = 0; al < 4; ++al)
            r.s[al] = b.s[al] - d.s[al];
    }

    for (int stp = 0; stp < nmr; ++stp) {
        if (active) {
#pragma unroll
            for (int al = 0; al < 4; ++al)
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    lr[(3 * al + a) * Vsb + t] = r.s[al].c[a];
        }
        __syncthreads();
        // acc = -2 D_Lambda r: it starts at -2 diag r and collects the inside
        // hops, so the MR coefficient follows from it without forming D_Lambda r
        spinor<float> acc;
        // the lane's products summed in FP32, the block sums in FP64
        float fr_re = 0.0f, fr_im = 0.0f, fqq = 0.0f;
        if (active) {
#pragma unroll
            for (int al = 0; al < 4; ++al)
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    acc.s[al].c[a] = cpx<float>{-2.0f * diag * r.s[al].c[a].re, -2.0f * diag * r.s[al].c[a].im};
#pragma unroll
            for (int h = 0; h < 8; ++h) {
                const int mu = h >> 1;
                const int step = (h & 1) ? -1 : +1;
                if (step > 0 ? yl[mu] + 1 < sbl[mu] : yl[mu] > 0) {
                    const int tn = t + step * lst[mu];
                    spinor<float> p;
#pragma unroll
                    for (int al = 0; al < 4; ++al)
#pragma unroll
                        for (int a = 0; a < 3; ++a)
                            p.s[al].c[a] = lr[(3 * al + a) * Vsb + tn];
                    const su3<float> u = expand_lds(lk[h], l3 + 3 * h * Vsb + t, Vsb);
                    if (step > 0)
                        hop_fwd_rt(mu, u, p, acc);
                    else
                        hop_bwd_rt(mu, u, p, acc);
                }
                if (h & 1)
                    asm volatile("" ::: "memory");
            }
#pragma unroll
            for (int al = 0; al < 4; ++al)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const float qa = acc.s[al].c[a].re, qb = acc.s[al].c[a].im;
                    const float ra = r.s[al].c[a].re, rb = r.s[al].c[a].im;
                    fr_re = fmadd(qb, rb, fmadd(qa, ra, fr_re));
                    fr_im = fmadd(-qb, ra, fmadd(qa, rb, fr_im));
                    fqq = fmadd(qb, qb, fmadd(qa, qa, fqq));
                }
        }
        const double qr_re = wave_sum((double)fr_re);
        const double qr_im = wave_sum((double)fr_im);
        const double qq = wave_sum((double)fqq);
        if (lane == 0) {
            red[0][wid] = qr_re;
            red[1][wid] = qr_im;
            red[2][wid] = qq;
        }
        __syncthreads();
        double sre = 0.0, sim = 0.0, sqq = 0.0;
        for (int w = 0; w < nw; ++w) {
            sre += red[0][w];
            sim += red[1][w];
            sqq += red[2][w];
        }
        if (!(sqq > 0.0))
            break;  // zero residue on this block: uniform across the workgroup
        // with q = D_Lambda r = -acc / 2: alpha = (q, r) / ||q||^2 = -2 (acc, r) / ||acc||^2,
        // x += alpha r, r -= alpha q = r + (alpha / 2) acc
        const c32 alpha{(float)(-2.0 * sre / sqq), (float)(-2.0 * sim / sqq)};
        const c32 half{0.5f * alpha.re, 0.5f * alpha.im};
#pragma unroll
        for (int al = 0; al < 4; ++al)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                xs.s[al].c[a] = cfma(alpha, r.s[al].c[a], xs.s[al].c[a]);
                r.s[al].c[a] = cfma(half, acc.s[al].c[a], r.s[al].c[a]);
            }
    }

    if (active) {
        spinor<float> p;
        zero(p);
        if (init == 0)
            p = load_spinor(psi, g.V, s);
#pragma unroll
        for (int al = 0; al < 4; ++al)
            p.s[al] += xs.s[al];
        store_spinor(psi, g.V, s, p);
        if (out64)
            store_spinor_f64(out64, g.V, s, p);
    }
}

// ---------------------------------------------------------------- lane pairs
//
// FP32 sweep with two lanes per site (adjacent lanes 2i, 2i+1). The even lane
// takes the four forward hops, (1 - g_mu) U_mu(x) psi(x + mu), the odd lane
// the four backward ones, (1 + g_mu) U_mu(x - mu)^+ psi(x - mu). The odd lane
// holds the adjoint of its link, and its spin projection and reconstruction
// equal the forward ones with the sign of every e_mu term flipped (see the
// projector identities in hop.h), so both lanes run one instruction stream
// with the sign as an FMA operand. The pair's partial sums are combined by
// one cross-lane add per real, and each lane owns two of the site's four spin
// components of the residue, the MR direction and the block solution
// (even: spins 0 and 1, odd: 2 and 3). Four links of 3x3 per lane (72 VGPRs)
// leave room for two wavefronts per SIMD.

// x + s*y, x + s*i*y and x - s*i*y with the lane's sign s
__device__ inline c32 add_s(c32 x, float sg, c32 y) { return {fmaf(sg, y.re, x.re), fmaf(sg, y.im, x.im)}; }
__device__ inline c32 add_si(c32 x, float sg, c32 y) { return {fmaf(-sg, y.im, x.re), fmaf(sg, y.re, x.im)}; }
__device__ inline c32 add_smi(c32 x, float sg, c32 y) { return {fmaf(sg, y.im, x.re), fmaf(-sg, y.re, x.im)}; }

// acc += forward (sg = +1, w = U_mu(x)) or backward (sg = -1, w = U_mu(x-mu)^+) hop of p
template <int MU>
__device__ inline void hop_pair(const su3<float>& w, const spinor<float>& p, float sg, spinor<float>& acc)
{
    cvec3<float> h0, h1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (MU == 0) {
            h0.c[a] = add_s(p.s[0].c[a], sg, p.s[2].c[a]);
            h1.c[a] = add_s(p.s[1].c[a], sg, p.s[3].c[a]);
        } else if (MU == 1) {
            h0.c[a] = add_si(p.s[0].c[a], sg, p.s[3].c[a]);
            h1.c[a] = add_si(p.s[1].c[a], sg, p.s[2].c[a]);
        } else if (MU == 2) {
            h0.c[a] = add_s(p.s[0].c[a], sg, p.s[3].c[a]);
            h1.c[a] = add_s(p.s[1].c[a], -sg, p.s[2].c[a]);
        } else {
            h0.c[a] = add_si(p.s[0].c[a], sg, p.s[2].c[a]);
            h1.c[a] = add_smi(p.s[1].c[a], sg, p.s[3].c[a]);
        }
    }
    cvec3<float> w0 = mul(w, h0);
    cvec3<float> w1 = mul(w, h1);
    acc.s[0] += w0;
    acc.s[1] += w1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (MU == 0) {
            acc.s[2].c[a] = add_s(acc.s[2].c[a], sg, w0.c[a]);
            acc.s[3].c[a] = add_s(acc.s[3].c[a], sg, w1.c[a]);
        } else if (MU == 1) {
            acc.s[2].c[a] = add_smi(acc.s[2].c[a], sg, w1.c[a]);
            acc.s[3].c[a] = add_smi(acc.s[3].c[a], sg, w0.c[a]);
        } else if (MU == 2) {
            acc.s[2].c[a] = add_s(acc.s[2].c[a], -sg, w1.c[a]);
            acc.s[3].c[a] = add_s(acc.s[3].c[a], sg, w0.c[a]);
        } else {
            acc.s[2].c[a] = add_smi(acc.s[2].c[a], sg, w0.c[a]);
            acc.s[3].c[a] = add_si(acc.s[3].c[a], sg, w1.c[a]);
        }
    }
}

// v + (v of the other lane of the pair); every lane of the wavefront must take part
__device__ inline float pair_sum(float v)
{
    // DPP quad_perm [1, 0, 3, 2]: swap adjacent lanes
    int o = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false);
    return v + __int_as_float(o);
}

// the lane's link for direction mu: U_mu(x) (forward lane) or U_mu(x - mu)^+ (backward lane)
template <typename L> __device__ inline su3<float> pair_link(const L& U, int mu, long site, bool bwd)
{
    su3<float> u = expand(load_link2(U, mu, site));
    su3<float> w;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const c32 x = u.m[a][b], y = u.m[b][a];
            w.m[a][b] = bwd ? c32{y.re, -y.im} : x;
        }
    return w;
}

template <typename L>
__global__ __launch_bounds__(512, 1) void k_sap_pair(Geom g, SapGeom sg, L U, const c32* __restrict__ rho,
                                                     const double* __restrict__ rho_nrm2, c32* __restrict__ psi,
                                                     float diag, int nmr, int colour, int nrhs, int init,
                                                     c64* __restrict__ out64)
{
    const float rs = rho_scale<float>(rho_nrm2, blockIdx.x % nrhs);
    rho += (long)(blockIdx.x % nrhs) * 12 * g.V;
    psi += (long)(blockIdx.x % nrhs) * 12 * g.V;
    if (out64)
        out64 += (long)(blockIdx.x % nrhs) * 12 * g.V;
    extern __shared__ char smem_raw[];
    c32* lr = reinterpret_cast<c32*>(smem_raw);
    __shared__ double red[3][8];

    const int t = threadIdx.x;
    const int ts = t >> 1;           // site in the block
    const int hb = t & 1;            // 0: forward hops, spins 0-1; 1: backward hops, spins 2-3
    const float sgn = hb ? -1.0f : 1.0f;
    const bool active = ts < sg.Vsb;  // both lanes of a pair agree
    const int lane = t & 63, wid = t >> 6, nw = blockDim.x >> 6;

    int k = blockIdx.x / nrhs;
    int half = sg.nsb[3] / 2;
    int m[4];
    int j = k % half;
    int rest = k / half;
    m[2] = rest % sg.nsb[2];
    rest /= sg.nsb[2];
    m[1] = rest % sg.nsb[1];
    m[0] = rest / sg.nsb[1];
    m[3] = 2 * j + ((colour + m[0] + m[1] + m[2]) & 1);

    int yl[4] = {0, 0, 0, 0};
    int n[4] = {0, 0, 0, 0}, y[4] = {0, 0, 0, 0};
    long s = 0;
    if (active) {
        int tt = ts;
        yl[3] = tt % sg.sb[3];
        tt /= sg.sb[3];
        yl[2] = tt % sg.sb[2];
        tt /= sg.sb[2];
        yl[1] = tt % sg.sb[1];
        yl[0] = tt / sg.sb[1];
        for (int mu = 0; mu < 4; ++mu) {
            int x = m[mu] * sg.sb[mu] + yl[mu];
            n[mu] = x / g.b[mu];
            y[mu] = x - n[mu] * g.b[mu];
        }
        s = site_compose(g, n, y);
    }
    // neighbour of this lane's hop inside the block
    bool inside[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
        inside[mu] = hb ? yl[mu] > 0 : yl[mu] + 1 < sg.sb[mu];
    const int c0 = 6 * hb;  // first owned component (3 * spin + colour)

    // residual with the full operator; the links are kept for the MR steps
    su3<float> lk[4];
    spinor<float> acc;
    zero(acc);
    if (active) {
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            long tn = site_step(g, s, n, y, mu, hb ? -1 : +1);
            lk[mu] = pair_link(U, mu, hb ? tn : s, hb != 0);
            if (init == 0 || (init == 1 && !inside[mu])) {
                spinor<float> p = load_spinor(psi, g.V, tn);
                if (mu == 0) hop_pair<0>(lk[0], p, sgn, acc);
                else if (mu == 1) hop_pair<1>(lk[1], p, sgn, acc);
                else if (mu == 2) hop_pair<2>(lk[2], p, sgn, acc);
                else hop_pair<3>(lk[3], p, sgn, acc);
            }
            if (mu & 1)
                asm volatile("" ::: "memory");  // two hops' loads in flight at a time
        }
    }
    c32 r[6], xs[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        // pair sum, then the owned half (spins 0-1 or 2-3)
        const int al = i / 3, a = i % 3;
        c32 lo{pair_sum(acc.s[al].c[a].re), pair_sum(acc.s[al].c[a].im)};
        c32 hi{pair_sum(acc.s[al + 2].c[a].re), pair_sum(acc.s[al + 2].c[a].im)};
        c32 ao = hb ? hi : lo;
        r[i] = c32{0.0f, 0.0f};
        xs[i] = c32{0.0f, 0.0f};
        if (active) {
            c32 self = c32{0.0f, 0.0f};
            if (init == 0)
                self = ld(psi, toff<c32>(s, c0 + i, 12));
            c32 b = ld(rho, toff<c32>(s, c0 + i, 12));
            if (rho_nrm2)
                b = c32{b.re * rs, b.im * rs};
            r[i] = c32{b.re - (diag * self.re - 0.5f * ao.re), b.im - (diag * self.im - 0.5f * ao.im)};
        }
    }

    for (int stp = 0; stp < nmr; ++stp) {
        if (active) {
#pragma unroll
            for (int i = 0; i < 6; ++i)
                lr[(c0 + i) * sg.Vsb + ts] = r[i];
        }
        __syncthreads();
        zero(acc);
        if (active) {
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) {
                if (inside[mu]) {
                    const int tn = ts + (hb ? -sg.lstr[mu] : sg.lstr[mu]);
                    spinor<float> p;
#pragma unroll
                    for (int al = 0; al < 4; ++al)
#pragma unroll
                        for (int a = 0; a < 3; ++a)
                            p.s[al].c[a] = lr[(3 * al + a) * sg.Vsb + tn];
                    if (mu == 0) hop_pair<0>(lk[0], p, sgn, acc);
                    else if (mu == 1) hop_pair<1>(lk[1], p, sgn, acc);
                    else if (mu == 2) hop_pair<2>(lk[2], p, sgn, acc);
                    else hop_pair<3>(lk[3], p, sgn, acc);
                }
                if (mu & 1)
                    asm volatile("" ::: "memory");
            }
        }
        c32 q[6];
        // the lane's products summed in FP32, the block sums in FP64
        float fr_re = 0.0f, fr_im = 0.0f, fqq = 0.0f;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const int al = i / 3, a = i % 3;
            c32 lo{pair_sum(acc.s[al].c[a].re), pair_sum(acc.s[al].c[a].im)};
            c32 hi{pair_sum(acc.s[al + 2].c[a].re), pair_sum(acc.s[al + 2].c[a].im)};
            c32 ao = hb ? hi : lo;
            q[i] = c32{diag * r[i].re - 0.5f * ao.re, diag * r[i].im - 0.5f * ao.im};
            const float qa = q[i].re, qb = q[i].im;
            const float ra = r[i].re, rb = r[i].im;
            fr_re = fmadd(qb, rb, fmadd(qa, ra, fr_re));
            fr_im = fmadd(-qb, ra, fmadd(qa, rb, fr_im));
            fqq = fmadd(qb, qb, fmadd(qa, qa, fqq));
        }
        const double qr_re = wave_sum((double)fr_re);
        const double qr_im = wave_sum((double)fr_im);
        const double qq = wave_sum((double)fqq);
        if (lane == 0) {
            red[0][wid] = qr_re;
            red[1][wid] = qr_im;
            red[2][wid] = qq;
        }
        __syncthreads();
        double sre = 0.0, sim = 0.0, sqq = 0.0;
        for (int w = 0; w < nw; ++w) {
            sre += red[0][w];
            sim += red[1][w];
            sqq += red[2][w];
        }
        if (!(sqq > 0.0))
            break;  // zero residue on this block: uniform across the workgroup
        c32 alpha{(float)(sre / sqq), (float)(sim / sqq)};
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            xs[i] = cfma(alpha, r[i], xs[i]);
            r[i] = cfma(-alpha, q[i], r[i]);
        }
    }

    if (active) {
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            c32 p = xs[i];
            if (init == 0)
                p += ld(psi, toff<c32>(s, c0 + i, 12));
            st(psi, toff<c32>(s, c0 + i, 12), p);
            if (out64)
                st(out64, toff<c64>(s, c0 + i, 12), c64{(double)p.re, (double)p.im});
        }
    }
}

template <typename T, typename L>
void launch(const Geom& g, const SapGeom& sg, L U, const cpx<T>* rho, const double* rho_nrm2, cpx<T>* psi, T m0,
            int nmr, int colour, int nrhs, int init, c64* out64, hipStream_t s, const cpx<T>* clov);

// Blocks of up to 256 sites: links in registers. One field on lattices whose
// colours hold few blocks per CU (sg.one_rl == 0): lane pairs, one block per
// CU at two wavefronts per SIMD (16^4 and 32 x 16^3 with 4^4 blocks: 11%
// faster than one lane per site); several fields, or one field with many
// blocks per colour: one lane per site, two blocks per CU (16 fields on 16^4:
// 12% faster than the generic kernel at three blocks per CU, which re-reads
// the links every MR step, and 28% faster than lane pairs; one field on
// 64 x 32^3: 346 against 475 us per sweep with lane pairs).
// Larger blocks, the clover term and antiperiodic time: the generic kernel.
template <typename L>
void launch_rl(const Geom& g, const SapGeom& sg, L U, const c32* rho, const double* rho_nrm2, c32* psi, float m0,
               int nmr, int colour, int nrhs, int init, c64* out64, hipStream_t s, const c32* clov)
{
    if (sg.Vsb > 256 || clov || g.tsign < 0) {
        launch<float, L>(g, sg, U, rho, rho_nrm2, psi, m0, nmr, colour, nrhs, init, out64, s, clov);
        return;
    }
    size_t lds = (size_t)12 * sg.Vsb * sizeof(c32);
    if (nrhs == 1 && !sg.one_rl) {
        int threads = ((2 * sg.Vsb + 63) / 64) * 64;
        hipLaunchKernelGGL((k_sap_pair<L>), dim3(sg.n_per_colour * nrhs), dim3(threads), lds, s, g, sg, U, rho,
                           rho_nrm2, psi, 4.0f + m0, nmr, colour, nrhs, init, out64);
        return;
    }
    int threads = ((sg.Vsb + 63) / 64) * 64;
    size_t lds_rl = (size_t)36 * sg.Vsb * sizeof(c32);
    static std::once_flag attr;  // one per link type
    static std::once_flag attr4;
    const bool b4 = sg.sb[0] == 4 && sg.sb[1] == 4 && sg.sb[2] == 4 && sg.sb[3] == 4;
    if (b4) {
        set_max_lds_once(attr4, reinterpret_cast<const void*>(&k_sap_rl<L, true>), 80 * 1024);
        hipLaunchKernelGGL((k_sap_rl<L, true>), dim3(sg.n_per_colour * nrhs), dim3(threads), lds_rl, s, g, sg, U,
                           rho, rho_nrm2, psi, 4.0f + m0, nmr, colour, nrhs, init, out64);
    } else {
        set_max_lds_once(attr, reinterpret_cast<const void*>(&k_sap_rl<L, false>), 80 * 1024);
        hipLaunchKernelGGL((k_sap_rl<L, false>), dim3(sg.n_per_colour * nrhs), dim3(threads), lds_rl, s, g, sg, U,
                           rho, rho_nrm2, psi, 4.0f + m0, nmr, colour, nrhs, init, out64);
    }
}

template <typename T, typename L>
void launch(const Geom& g, const SapGeom& sg, L U, const cpx<T>* rho, const double* rho_nrm2, cpx<T>* psi, T m0,
            int nmr, int colour, int nrhs, int init, c64* out64, hipStream_t s, const cpx<T>* clov)
{
    int threads = ((sg.Vsb + 63) / 64) * 64;
    size_t lds = (size_t)12 * sg.Vsb * sizeof(cpx<T>);
    const Clover<T> C{clov};
    if (clov) {
        static std::once_flag attr;  // one per kernel instantiation
        set_max_lds_once(attr, reinterpret_cast<const void*>(&k_sap<T, L, true>), 160 * 1024 - 1024);
        hipLaunchKernelGGL((k_sap<T, L, true>), dim3(sg.n_per_colour * nrhs), dim3(threads), lds, s, g, sg, U, rho,
                           rho_nrm2, psi, T(4) + m0, nmr, colour, nrhs, init, out64, C);
    } else {
        static std::once_flag attr;
        set_max_lds_once(attr, reinterpret_cast<const void*>(&k_sap<T, L, false>), 160 * 1024 - 1024);
        hipLaunchKernelGGL((k_sap<T, L, false>), dim3(sg.n_per_colour * nrhs), dim3(threads), lds, s, g, sg, U, rho,
                           rho_nrm2, psi, T(4) + m0, nmr, colour, nrhs, init, out64, C);
    }
}

}  // namespace

void launch_sap_colour64(const Geom& g, const SapGeom& sg, Links64 U, const c64* rho, c64* psi, double m0, int nmr,
                         int colour, int nrhs, int init, hipStream_t s, const c64* clov)
{
    launch(g, sg, U, rho, (const double*)nullptr, psi, m0, nmr, colour, nrhs, init, (c64*)nullptr, s, clov);
}
void launch_sap_colour32(const Geom& g, const SapGeom& sg, Links32 U, const c32* rho, c32* psi, float m0, int nmr,
                         int colour, int nrhs, int init, c64* out64, hipStream_t s, const c32* clov,
                         const double* rho_nrm2)
{
    launch_rl(g, sg, U, rho, rho_nrm2, psi, m0, nmr, colour, nrhs, init, out64, s, clov);
}
void launch_sap_colour_bf16(const Geom& g, const SapGeom& sg, LinksBF16 U, const c32* rho, c32* psi, float m0,
                            int nmr, int colour, int nrhs, int init, c64* out64, hipStream_t s, const c32* clov,
                            const double* rho_nrm2)
{
    launch_rl(g, sg, U, rho, rho_nrm2, psi, m0, nmr, colour, nrhs, init, out64, s, clov);
}

}  // namespace dfl
