/*
 * FP64 CPU oracle: Wilson-Dirac stencil, block-restricted operator, Schwarz
 * alternating procedure.
 *
 * TEST INFRASTRUCTURE ONLY. This file is compiled into liboracle.so and is
 * used by the tests, by the smoke check and by the CPU-baseline leg of the
 * benchmark. The HIP library never links, loads or calls it, and it shares no
 * code, header or table with the HIP library.
 *
 * Everything is plain FP64 (C99 double complex), written for a reader who
 * checks it against the paper by eye: one loop per sum in the definition, no
 * blocking, no spin-projection shortcut, no reordering.
 *
 * Canonical layout (the same as the synthetic-input generator):
 *   site s = ((x0*L1 + x1)*L2 + x2)*L3 + x3, x0 slowest;
 *   quark field psi[s*12 + 3*alpha + a] (spin alpha, colour a);
 *   gauge field U[((s*4 + mu)*3 + a)*3 + b], the link x -> x+mu.
 *
 * Operator (the paper's D of eq. (3.9): the Wilson operator with the
 * O(a)-improvement term of section 2.1, chiral gamma basis):
 *   (D psi)(x) = (4 + m0) psi(x) + csw (i/4) sum_{mu,nu} sigma_{mu nu} Fhat_{mu nu}(x) psi(x)
 *       - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)
 *                    + (1 + g_mu) U_mu(x-mu)^dagger psi(x-mu) ].
 * gamma_mu = [[0, e_mu], [e_mu^dagger, 0]] with e_0 = -1, e_k = -i sigma_k;
 * sigma_{mu nu} = (i/2)[g_mu, g_nu]; Fhat_{mu nu}(x) = (Q_{mu nu}(x) - Q_{nu mu}(x))/8
 * with Q_{mu nu}(x) the sum of the four plaquettes in the (mu, nu) plane that
 * start and end at x (the "clover leaves"). csw = 0 is the plain Wilson
 * operator. Boundary conditions: periodic in space; in time (direction 0)
 * periodic (bc0 = +1) or antiperiodic (bc0 = -1: a hop across the time
 * boundary x0 = L0-1 <-> 0 carries a factor -1).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ---------------------------------------------------------------- gamma */

static cplx GAMMA[4][4][4];
static int gamma_ready = 0;

static void init_gamma(void)
{
    if (gamma_ready)
        return;
    /* e_mu as 2x2 blocks */
    cplx e[4][2][2];
    memset(e, 0, sizeof(e));
    e[0][0][0] = -1.0;
    e[0][1][1] = -1.0;
    /* e_1 = -i sigma_1 */
    e[1][0][1] = -I;
    e[1][1][0] = -I;
    /* e_2 = -i sigma_2, sigma_2 = [[0,-i],[i,0]] */
    e[2][0][1] = -1.0;
    e[2][1][0] = 1.0;
    /* e_3 = -i sigma_3 */
    e[3][0][0] = -I;
    e[3][1][1] = I;
    memset(GAMMA, 0, sizeof(GAMMA));
    for (int mu = 0; mu < 4; ++mu)
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                GAMMA[mu][i][2 + j] = e[mu][i][j];        /* upper right: e_mu */
                GAMMA[mu][2 + i][j] = conj(e[mu][j][i]);  /* lower left: e_mu^dagger */
            }
    gamma_ready = 1;
}

/* Export the gamma matrices so tests can check the Clifford algebra. */
void orc_gamma(double *out /* [4][4][4] complex */)
{
    init_gamma();
    memcpy(out, GAMMA, sizeof(GAMMA));
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------- geometry */

static void site_coords(const int L[4], long s, int x[4])
{
    x[3] = (int)(s % L[3]);
    s /= L[3];
    x[2] = (int)(s % L[2]);
    s /= L[2];
    x[1] = (int)(s % L[1]);
    x[0] = (int)(s / L[1]);
}

static long site_index(const int L[4], const int x[4])
{
    return (((long)x[0] * L[1] + x[1]) * L[2] + x[2]) * L[3] + x[3];
}

static long site_shift(const int L[4], long s, int mu, int step)
{
    int x[4];
    site_coords(L, s, x);
    x[mu] = ((x[mu] + step) % L[mu] + L[mu]) % L[mu];
    return site_index(L, x);
}

/* Block index of site s for block shape b: lexicographic over block coords. */
static long block_of(const int L[4], const int b[4], long s)
{
    int x[4];
    site_coords(L, s, x);
    long k = 0;
    for (int mu = 0; mu < 4; ++mu)
        k = k * (L[mu] / b[mu]) + x[mu] / b[mu];
    return k;
}

/* --------------------------------------------------------- hop terms */

/* -1 for a hop across the time boundary with antiperiodic time (bc0 = -1) */
static double bc_sign(const int L[4], long s, int mu, int step, int bc0)
{
    if (mu != 0 || bc0 > 0)
        return 1.0;
    int x[4];
    site_coords(L, s, x);
    if ((step > 0 && x[0] == L[0] - 1) || (step < 0 && x[0] == 0))
        return -1.0;
    return 1.0;
}

/* out(x) += -1/2 (1 - g_mu) U_mu(x) psi(x+mu)   (forward hop) */
static void hop_forward(const int L[4], const cplx *U, const cplx *psi, long s, int mu, int bc0, cplx *out)
{
    long t = site_shift(L, s, mu, +1);
    double sg = bc_sign(L, s, mu, +1, bc0);
    const cplx *u = U + (s * 4 + mu) * 9;
    cplx chi[4][3];
    for (int al = 0; al < 4; ++al)
        for (int a = 0; a < 3; ++a) {
            cplx acc = 0;
            for (int b = 0; b < 3; ++b)
                acc += u[a * 3 + b] * psi[t * 12 + 3 * al + b];
            chi[al][a] = acc;
        }
    for (int al = 0; al < 4; ++al)
        for (int a = 0; a < 3; ++a) {
            cplx gchi = 0;
            for (int be = 0; be < 4; ++be)
                gchi += GAMMA[mu][al][be] * chi[be][a];
            out[3 * al + a] += -0.5 * sg * (chi[al][a] - gchi);
        }
}

/* out(x) += -1/2 (1 + g_mu) U_mu(x-mu)^dagger psi(x-mu)   (backward hop) */
static void hop_backward(const int L[4], const cplx *U, const cplx *psi, long s, int mu, int bc0, cplx *out)
{
    long t = site_shift(L, s, mu, -1);
    double sg = bc_sign(L, s, mu, -1, bc0);
    const cplx *u = U + (t * 4 + mu) * 9;
    cplx chi[4][3];
    for (int al = 0; al < 4; ++al)
        for (int a = 0; a < 3; ++a) {
            cplx acc = 0;
            for (int b = 0; b < 3; ++b)
                acc += conj(u[b * 3 + a]) * psi[t * 12 + 3 * al + b];
            chi[al][a] = acc;
        }
    for (int al = 0; al < 4; ++al)
        for (int a = 0; a < 3; ++a) {
            cplx gchi = 0;
            for (int be = 0; be < 4; ++be)
                gchi += GAMMA[mu][al][be] * chi[be][a];
            out[3 * al + a] += -0.5 * sg * (chi[al][a] + gchi);
        }
}

/* ---------------------------------------------------------- clover term */

/* c = a b (3x3); ad/bd: use the adjoint of a / b */
static void mat3_mul(const cplx *a, int ad, const cplx *b, int bd, cplx *c)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx acc = 0;
            for (int k = 0; k < 3; ++k) {
                cplx x = ad ? conj(a[k * 3 + i]) : a[i * 3 + k];
                cplx y = bd ? conj(b[j * 3 + k]) : b[k * 3 + j];
                acc += x * y;
            }
            c[i * 3 + j] = acc;
        }
}

/* product of four links l[0] l[1] l[2] l[3], each taken as given or adjoint */
static void path4(const cplx *l[4], const int dag[4], cplx *out)
{
    cplx t1[9], t2[9];
    mat3_mul(l[0], dag[0], l[1], dag[1], t1);
    mat3_mul(t1, 0, l[2], dag[2], t2);
    mat3_mul(t2, 0, l[3], dag[3], out);
}

static const cplx *link(const cplx *U, long s, int mu) { return U + (s * 4 + mu) * 9; }

/*
 * Fhat_{mu nu}(x) = (Q_{mu nu} - Q_{mu nu}^dagger) / 8 with the four leaves
 *   U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
 *   U_nu(x) U_mu(x+nu-mu)^+ U_nu(x-mu)^+ U_mu(x-mu)
 *   U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
 *   U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^+
 * (Q_{nu mu} = Q_{mu nu}^dagger: the same leaves run the other way round).
 */
static void field_tensor(const int L[4], const cplx *U, long s, int mu, int nu, cplx F[9])
{
    long xpm = site_shift(L, s, mu, +1), xpn = site_shift(L, s, nu, +1);
    long xmm = site_shift(L, s, mu, -1), xmn = site_shift(L, s, nu, -1);
    long xmm_pn = site_shift(L, xmm, nu, +1), xmm_mn = site_shift(L, xmm, nu, -1);
    long xmn_pm = site_shift(L, xmn, mu, +1);
    cplx Q[9] = {0}, leaf[9];
    const cplx *l1[4] = {link(U, s, mu), link(U, xpm, nu), link(U, xpn, mu), link(U, s, nu)};
    const int d1[4] = {0, 0, 1, 1};
    const cplx *l2[4] = {link(U, s, nu), link(U, xmm_pn, mu), link(U, xmm, nu), link(U, xmm, mu)};
    const int d2[4] = {0, 1, 1, 0};
    const cplx *l3[4] = {link(U, xmm, mu), link(U, xmm_mn, nu), link(U, xmm_mn, mu), link(U, xmn, nu)};
    const int d3[4] = {1, 1, 0, 0};
    const cplx *l4[4] = {link(U, xmn, nu), link(U, xmn, mu), link(U, xmn_pm, nu), link(U, s, mu)};
    const int d4[4] = {1, 0, 0, 1};
    const cplx **ls[4] = {l1, l2, l3, l4};
    const int *ds[4] = {d1, d2, d3, d4};
    for (int q = 0; q < 4; ++q) {
        path4(ls[q], ds[q], leaf);
        for (int i = 0; i < 9; ++i)
            Q[i] += leaf[i];
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            F[i * 3 + j] = (Q[i * 3 + j] - conj(Q[j * 3 + i])) / 8.0;
}

/* C(x) = csw (i/4) sum_{mu != nu} sigma_{mu nu} (x) Fhat_{mu nu}(x), index 3 alpha + a */
static void clover_site(const int L[4], const cplx *U, double csw, long s, cplx C[12][12])
{
    memset(C, 0, sizeof(cplx) * 144);
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu) {
            if (mu == nu)
                continue;
            cplx F[9];
            field_tensor(L, U, s, mu, nu, F);
            for (int al = 0; al < 4; ++al)
                for (int be = 0; be < 4; ++be) {
                    /* sigma_{mu nu} = (i/2) (g_mu g_nu - g_nu g_mu) */
                    cplx sig = 0;
                    for (int ga = 0; ga < 4; ++ga)
                        sig += GAMMA[mu][al][ga] * GAMMA[nu][ga][be] - GAMMA[nu][al][ga] * GAMMA[mu][ga][be];
                    sig *= 0.5 * I;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b)
                            C[3 * al + a][3 * be + b] += csw * 0.25 * I * sig * F[a * 3 + b];
                }
        }
}

/* out += C(x) psi(x) */
static void clover_add(const int L[4], const cplx *U, double csw, const cplx *psi, long s, cplx *out)
{
    if (csw == 0.0)
        return;
    cplx C[12][12];
    clover_site(L, U, csw, s, C);
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j)
            out[i] += C[i][j] * psi[s * 12 + j];
}

/* The clover matrix of site s (for the tests), [12][12] complex. */
void orc_clover_site(const int L[4], const cplx *U, double csw, long s, cplx *out)
{
    init_gamma();
    cplx C[12][12];
    clover_site(L, U, csw, s, C);
    memcpy(out, C, sizeof(C));
}

/*
 * Generic stencil. mode selects which hops are kept:
 *   0: all hops (full D, eq. (3.9));
 *   1: only hops whose both ends lie in the same block of shape b
 *      (block-diagonal part, the direct sum of the D_Lambda);
 *   2: only hops that leave the block, in one direction mu and one
 *      orientation dir (+1 forward / -1 backward), no mass term.
 * The mass term (4+m0) psi(x) is included in modes 0 and 1.
 */
static void stencil(const int L[4], const int *b, double m0, double csw, int bc0, const cplx *U,
                    const cplx *psi, cplx *out, int mode, int hop_mu, int hop_dir)
{
    init_gamma();
    long V = (long)L[0] * L[1] * L[2] * L[3];
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        cplx acc[12];
        for (int c = 0; c < 12; ++c)
            acc[c] = (mode == 2) ? 0.0 : (4.0 + m0) * psi[s * 12 + c];
        if (mode != 2)
            clover_add(L, U, csw, psi, s, acc);
        for (int mu = 0; mu < 4; ++mu) {
            long fwd = site_shift(L, s, mu, +1);
            long bwd = site_shift(L, s, mu, -1);
            int keep_f = 1, keep_b = 1;
            if (mode == 1) {
                keep_f = block_of(L, b, fwd) == block_of(L, b, s);
                keep_b = block_of(L, b, bwd) == block_of(L, b, s);
            } else if (mode == 2) {
                keep_f = (mu == hop_mu && hop_dir > 0) && block_of(L, b, fwd) != block_of(L, b, s);
                keep_b = (mu == hop_mu && hop_dir < 0) && block_of(L, b, bwd) != block_of(L, b, s);
            }
            if (keep_f)
                hop_forward(L, U, psi, s, mu, bc0, acc);
            if (keep_b)
                hop_backward(L, U, psi, s, mu, bc0, acc);
        }
        for (int c = 0; c < 12; ++c)
            out[s * 12 + c] = acc[c];
    }
}

/* out = D psi on the whole lattice. */
void orc_dirac(const int L[4], double m0, double csw, int bc0, const cplx *U, const cplx *psi, cplx *out)
{
    stencil(L, NULL, m0, csw, bc0, U, psi, out, 0, 0, 0);
}

/* out = (direct sum over blocks of D_Lambda) psi: hops across block faces dropped. */
void orc_dirac_blockdiag(const int L[4], const int b[4], double m0, double csw, int bc0, const cplx *U,
                         const cplx *psi, cplx *out)
{
    stencil(L, b, m0, csw, bc0, U, psi, out, 1, 0, 0);
}

/* out = the block-crossing hop terms of D in direction mu, orientation dir (+1/-1). */
void orc_hop_cross(const int L[4], const int b[4], int bc0, const cplx *U, const cplx *psi,
                   cplx *out, int mu, int dir)
{
    stencil(L, b, 0.0, 0.0, bc0, U, psi, out, 2, mu, dir);
}

/* (D psi)(x) for an explicit list of sites only: out[i*12 + c] for site sites[i]. */
void orc_dirac_sites(const int L[4], double m0, double csw, int bc0, const cplx *U, const cplx *psi,
                     const long *sites, long n, cplx *out)
{
    init_gamma();
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        long s = sites[i];
        cplx acc[12];
        for (int c = 0; c < 12; ++c)
            acc[c] = (4.0 + m0) * psi[s * 12 + c];
        clover_add(L, U, csw, psi, s, acc);
        for (int mu = 0; mu < 4; ++mu) {
            hop_forward(L, U, psi, s, mu, bc0, acc);
            hop_backward(L, U, psi, s, mu, bc0, acc);
        }
        for (int c = 0; c < 12; ++c)
            out[i * 12 + c] = acc[c];
    }
}

/* ------------------------------------------------------------ SAP */

/*
 * D_Lambda restricted to one block: out(x) for x in the block, using psi only
 * on the block (hops leaving the block are dropped, i.e. Dirichlet walls).
 * sites[] lists the block's sites, n of them; in/out are full-volume arrays and
 * only the block's entries are read or written.
 */
static void apply_dlambda(const int L[4], const int b[4], double m0, double csw, int bc0, const cplx *U,
                          const long *sites, long n, const cplx *in, cplx *out)
{
    for (long i = 0; i < n; ++i) {
        long s = sites[i];
        long blk = block_of(L, b, s);
        cplx acc[12];
        for (int c = 0; c < 12; ++c)
            acc[c] = (4.0 + m0) * in[s * 12 + c];
        clover_add(L, U, csw, in, s, acc);
        for (int mu = 0; mu < 4; ++mu) {
            if (block_of(L, b, site_shift(L, s, mu, +1)) == blk)
                hop_forward(L, U, in, s, mu, bc0, acc);
            if (block_of(L, b, site_shift(L, s, mu, -1)) == blk)
                hop_backward(L, U, in, s, mu, bc0, acc);
        }
        for (int c = 0; c < 12; ++c)
            out[s * 12 + c] = acc[c];
    }
}

/* (u, v) = sum conj(u) v over the block's sites */
static cplx block_dot(const long *sites, long n, const cplx *u, const cplx *v)
{
    cplx acc = 0;
    for (long i = 0; i < n; ++i)
        for (int c = 0; c < 12; ++c)
            acc += conj(u[sites[i] * 12 + c]) * v[sites[i] * 12 + c];
    return acc;
}

/*
 * Minimal-residual iteration for D_Lambda x = rhs on one block, nmr steps,
 * zero start: r = rhs; repeat { q = D_Lambda r; alpha = (q,r)/(q,q);
 * x += alpha r; r -= alpha q }. x and r/q scratch are full-volume arrays.
 */
static void mr_block(const int L[4], const int b[4], double m0, double csw, int bc0, const cplx *U,
                     const long *sites, long n, const cplx *rhs, int nmr,
                     cplx *x, cplx *r, cplx *q)
{
    for (long i = 0; i < n; ++i)
        for (int c = 0; c < 12; ++c) {
            x[sites[i] * 12 + c] = 0;
            r[sites[i] * 12 + c] = rhs[sites[i] * 12 + c];
        }
    for (int k = 0; k < nmr; ++k) {
        apply_dlambda(L, b, m0, csw, bc0, U, sites, n, r, q);
        double qq = creal(block_dot(sites, n, q, q));
        if (!(qq > 0.0))
            break;
        cplx alpha = block_dot(sites, n, q, r) / qq;
        for (long i = 0; i < n; ++i)
            for (int c = 0; c < 12; ++c) {
                long j = sites[i] * 12 + c;
                x[j] += alpha * r[j];
                r[j] -= alpha * q[j];
            }
    }
}

/* Public single-block MR (for the tests): x on the block sites of block blk. */
void orc_mr_block(const int L[4], const int b[4], double m0, double csw, int bc0, const cplx *U, long blk,
                  const cplx *rhs, int nmr, cplx *x)
{
    init_gamma();
    long V = (long)L[0] * L[1] * L[2] * L[3];
    long vb = (long)b[0] * b[1] * b[2] * b[3];
    long *sites = malloc(sizeof(long) * vb);
    long n = 0;
    for (long s = 0; s < V; ++s)
        if (block_of(L, b, s) == blk)
            sites[n++] = s;
    cplx *r = calloc((size_t)V * 12, sizeof(cplx));
    cplx *q = calloc((size_t)V * 12, sizeof(cplx));
    mr_block(L, b, m0, csw, bc0, U, sites, n, rhs, nmr, x, r, q);
    free(r);
    free(q);
    free(sites);
}

/*
 * Schwarz alternating procedure psi = M_sap rho (the preconditioner of eq. (6.2)):
 *   psi = 0;
 *   for ncy cycles, for colour 0 then colour 1:
 *     r = rho - D psi (full operator, so the hops from the neighbouring blocks
 *     enter through the current psi);
 *     on every block of that colour: psi_Lambda += MR_Lambda(r_Lambda, nmr).
 * Block colour = (sum of block coordinates) mod 2. Blocks of one colour share
 * no hop term, so they are independent and may be processed in any order.
 */
void orc_sap(const int L[4], const int b[4], double m0, double csw, int bc0, const cplx *U, const cplx *rho,
             int ncy, int nmr, cplx *psi)
{
    init_gamma();
    long V = (long)L[0] * L[1] * L[2] * L[3];
    int nb[4];
    long nblk = 1;
    for (int mu = 0; mu < 4; ++mu) {
        nb[mu] = L[mu] / b[mu];
        nblk *= nb[mu];
    }
    long vb = (long)b[0] * b[1] * b[2] * b[3];
    /* site lists per block, in canonical order */
    long *sites = malloc(sizeof(long) * V);
    long *fill = calloc((size_t)nblk, sizeof(long));
    for (long s = 0; s < V; ++s) {
        long k = block_of(L, b, s);
        sites[k * vb + fill[k]++] = s;
    }
    int *colour = malloc(sizeof(int) * nblk);
    for (long k = 0; k < nblk; ++k) {
        long t = k;
        int sum = 0;
        for (int mu = 3; mu >= 0; --mu) {
            sum += (int)(t % nb[mu]);
            t /= nb[mu];
        }
        colour[k] = sum % 2;
    }
    cplx *r = malloc(sizeof(cplx) * V * 12);
    cplx *x = malloc(sizeof(cplx) * V * 12);
    cplx *rr = malloc(sizeof(cplx) * V * 12);
    cplx *qq = malloc(sizeof(cplx) * V * 12);
    for (long j = 0; j < V * 12; ++j)
        psi[j] = 0;
    for (int cy = 0; cy < ncy; ++cy)
        for (int c = 0; c < 2; ++c) {
            orc_dirac(L, m0, csw, bc0, U, psi, r);
            for (long j = 0; j < V * 12; ++j)
                r[j] = rho[j] - r[j];
#pragma omp parallel for schedule(dynamic)
            for (long k = 0; k < nblk; ++k) {
                if (colour[k] != c)
                    continue;
                const long *sk = sites + k * vb;
                mr_block(L, b, m0, csw, bc0, U, sk, vb, r, nmr, x, rr, qq);
                for (long i = 0; i < vb; ++i)
                    for (int cc = 0; cc < 12; ++cc)
                        psi[sk[i] * 12 + cc] += x[sk[i] * 12 + cc];
            }
        }
    free(r);
    free(x);
    free(rr);
    free(qq);
    free(colour);
    free(fill);
    free(sites);
}
