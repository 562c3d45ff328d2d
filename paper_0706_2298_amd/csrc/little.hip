// GCR for the little system A v = w (eq. (6.1), appendix A.4) in a single
// cooperative launch.
//
// The little vector has Nb*Ns entries; workgroup g owns the blocks
// g, g + G, g + 2G, ... (G = grid size) and all entries of those blocks. One
// GCR step normally needs two grid-wide barriers (one more inside the
// even-odd operator):
//   S1  xi_k = r is complete everywhere: apply chi_k = A xi_k (rows of the
//       owned blocks; the nine neighbour blocks' entries are read from global
//       memory). Convergence is tested before it on ||r_k||^2 =
//       ||r_{k-1}||^2 - |c_k|^2, which needs no reduction;
//   S2  reduce (chi_j, chi_k), (chi_j, r) for j < k, ||chi_k||^2 and
//       (chi_k, r) in one pass; classical Gram-Schmidt then gives the
//       normalised chi_k, its coefficient c_k = (chi_k, r) and the new residue
//       without another reduction (||chi_k - sum a_j chi_j||^2 =
//       ||chi_k||^2 - sum |a_j|^2).
// If that single pass cancels more than 99% of ||chi_k||^2 (orthogonality
// would suffer), a second pass with its own barrier S3 repeats it.
// Partial sums are written per workgroup and every workgroup reduces them in
// the same fixed order, so all workgroups take identical decisions and the
// result is bit-reproducible. After nkv steps (or convergence) the solution
// is updated from the triangular system and the residue recomputed as
// w - A x (two more barriers); convergence is decided on that true residue. The barriers are this file's own (see
// grid_barrier); the launch is cooperative so all workgroups are resident.
#include "internal.h"

namespace dfl {

namespace {

constexpr int LT = 1024;            // threads per workgroup of the many-source solver (16 wavefronts)
constexpr int LT1 = 512;            // threads per workgroup of the single-source solver: a few blocks per
                                    // workgroup need no more, and 512 threads leave 256 VGPRs per lane
constexpr long kSpinLimit = 1L << 24;  // ~0.5 s of polling before a barrier gives up
constexpr int NK = kMaxLittleNkv;
// partial-sum slots
constexpr int NQ = kMaxLittleDefl;   // most global deflation directions of the little system
constexpr int SA = 0;                 // first pass: (chi_j, chi_k) j<k | (chi_j, r) j<k | ||chi_k||^2 | (chi_k, r) | (Q_l, chi_k)
constexpr int SB = 2 * NK + 2 + NQ;   // second pass, same layout
constexpr int SC = 2 * SB;            // ||r||^2 inside a cycle
constexpr int SR = SC + 1;            // ||r||^2 after a restart
constexpr int SW = SC + 2;            // ||w||^2
constexpr int SQ = SC + 3;            // (Q_l, r), or (Z_l, r) then (W_l, r), at the start and after a restart
constexpr int NSLOT = SQ + 2 * NQ;
static_assert(NK + NQ <= 64, "the coefficient step gives each projection one lane of a wavefront");

template <typename T> struct LittleArgs {
    Geom g;
    int Ns, nkv, maxiter;
    double tol2;           // stop at ||r||^2 <= tol2 * ||w||^2
    const double* tol_dev; // if set: the relative tolerance is read from here at entry
    const cpx<T>* At;      // [Nb][9][Ns(l)][Ns(k)]: transposed blocks
    const cpx<T>* Mt;      // even-odd: [Nb][0] = D^-1, [Nb][d] = D^-1 A_d, transposed likewise
    const cpx<T>* w;
    cpx<T>* x;
    cpx<T>* r;
    cpx<T>* xi;            // nkv * N
    cpx<T>* chi;           // nkv * N
    cpx<T>* w1;            // even-odd workspaces (N each)
    cpx<T>* w2;
    const cpx<T>* Q;       // global deflation (appendix A.3), minimal-residual form: nq orthonormal
    const cpx<T>* Z;       //   images Q = A_hat Z and their preimages Z, little vectors (even blocks);
                           //   oblique form: Q holds W = A_hat Z, Z is orthonormal
    int nq;
    int oblique;           // 1: the oblique projectors of section 3 on the even-odd system, with
    const double* Ainv;    //   Ainv = (Z^+ W)^-1 (nq x nq complex, row-major) and
    const double* Gw;      //   Gw = W^+ W (nq x nq complex)
    double* part;          // NSLOT * G complex partial sums, then NSLOT published sums
    int* stats;            // [0] += iterations, [1] += solves, [2] |= 1 not converged, |= 4 barrier timeout
    unsigned* bar_count;   // grid barrier: arrivals (0 between barriers)
    unsigned long long* bar_gen;  // grid barrier: generation, increases across launches
};

// Grid-wide barrier for a cooperative launch (all workgroups co-resident).
// Thread 0 of each workgroup publishes the workgroup's writes with one
// agent-scope release fence, counts in with a relaxed atomic, and (unless it
// is the last to arrive) polls the generation word with relaxed coherent
// loads; one agent-scope acquire fence follows. The last arrival resets the
// counter and publishes the next generation. Acquire/release semantics on
// every poll would make each poll an L2 invalidation, which serialises
// across the device; this form costs one cache write-back and one
// invalidation per workgroup and barrier. The generation word is never
// reset: a launch continues from the value the previous one left (read once
// at entry). Polling is bounded; on timeout the workgroup records a failure
// and continues, so every wave reaches the end.
__device__ inline void grid_barrier(unsigned* count, unsigned long long* gen, unsigned long long& target, int* stats)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        ++target;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        unsigned old = __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old == gridDim.x - 1) {
            __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(gen, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long spin = 0;
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(1);
                if (++spin > kSpinLimit) {
                    atomicOr(&stats[2], 4);
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

__device__ inline double2 cfma_conj(double2 acc, double ar, double ai, double br, double bi)
{
    // acc += conj(a) * b
    acc.x += ar * br + ai * bi;
    acc.y += ar * bi - ai * br;
    return acc;
}

constexpr int kMaxOwned = 1024;  // blocks one workgroup of the even-odd solver may own

// colour (sum of block coordinates mod 2) of block blk
__device__ inline int block_colour(const Geom& g, int blk)
{
    int sum = 0, rest = blk;
    for (int mu = 3; mu >= 0; --mu) {
        sum += rest % g.nb[mu];
        rest /= g.nb[mu];
    }
    return sum & 1;
}

__device__ inline int nbr_block(const Geom& g, int blk, int d)
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

// The workgroup's view: it owns the blocks g + i G (i = owned position); its
// vector entries are those of the owned positions listed in vb (all of them
// when vb is null). nbr (LDS, may be null): nbr[8 i + d - 1] = neighbour d of
// owned position i.
template <typename T> struct LittleCtx {
    const LittleArgs<T>& a;
    int G, g, t;
    long N;
    const int* vb;
    int nvb;
    const int* nbr;
    __device__ int block(int i) const { return g + (vb ? vb[i] : i) * G; }
    __device__ long entry(int e) const
    {
        int i = e / a.Ns;
        int k = e - i * a.Ns;
        return (long)block(i) * a.Ns + k;
    }
    __device__ int R() const { return nvb * a.Ns; }
};

// reduce slots [s0, s0 + ns) over the G workgroups into red (complex), identically everywhere
// Each wavefront reduces kSlotUnroll slots at a time so that their loads are
// in flight together (the partial sums were written by other workgroups and
// come from beyond the local L2).
constexpr int kSlotUnroll = 4;
__device__ inline void reduce_slots(const double* __restrict__ part, int G, int s0, int ns, double* red)
{
    constexpr int NW = LT1 / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int sb = w; sb < ns; sb += NW * kSlotUnroll) {
        double re[kSlotUnroll], im[kSlotUnroll];
#pragma unroll
        for (int u = 0; u < kSlotUnroll; ++u) {
            re[u] = 0.0;
            im[u] = 0.0;
        }
        // slots past ns read slot ns - 1 (valid memory, result dropped): no
        // branch separates the loads of the kSlotUnroll slots
        for (int q = lane; q < G; q += 64) {
            double2 v[kSlotUnroll];
#pragma unroll
            for (int u = 0; u < kSlotUnroll; ++u) {
                const int s = min(sb + u * NW, ns - 1);
                v[u] = *reinterpret_cast<const double2*>(part + ((long)(s0 + s) * G + q) * 2);
            }
#pragma unroll
            for (int u = 0; u < kSlotUnroll; ++u) {
                re[u] += v[u].x;
                im[u] += v[u].y;
            }
        }
#pragma unroll
        for (int u = 0; u < kSlotUnroll; ++u) {
            const int s = sb + u * NW;
            const double sr = wave_sum(re[u]), si = wave_sum(im[u]);
            if (s < ns && lane == 0) {
                red[2 * s] = sr;
                red[2 * s + 1] = si;
            }
        }
    }
    __syncthreads();
}

// Grid barrier that also reduces the partial-sum slots [s0, s0 + ns) over the
// G workgroups: the workgroup that arrives last sums them (reduce_slots, the
// same fixed order whichever workgroup it is, so the result is
// bit-reproducible), writes the ns complex sums to pub and only then publishes
// the next generation; the others wait for it and read the ns sums instead of
// all G ns partial sums. One workgroup thus reads the partials once, instead
// of every workgroup reading all of them from the other XCDs' L2. red: 2 ns
// doubles in LDS; last_s: an int in LDS. pub is not overwritten before every
// workgroup has read it (the next such barrier needs every workgroup's
// arrival first).
__device__ inline void grid_barrier_reduce(unsigned* count, unsigned long long* gen, unsigned long long& target,
                                           int* stats, const double* __restrict__ part, double* pub, int G, int s0,
                                           int ns, double* red, int* last_s)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        ++target;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned old = __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int last = old == gridDim.x - 1;
        if (last)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *last_s = last;
    }
    __syncthreads();
    if (*last_s) {
        reduce_slots(part, G, s0, ns, red);
        for (int q = threadIdx.x; q < 2 * ns; q += blockDim.x)
            pub[q] = red[q];
        __syncthreads();
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(gen, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        return;
    }
    if (threadIdx.x == 0) {
        long spin = 0;
        while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spin > kSpinLimit) {
                atomicOr(&stats[2], 4);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 2 * ns; q += blockDim.x)
        red[q] = pub[q];
    __syncthreads();
}

// y_blk = alpha s_blk + beta sum_{d0 <= d < d1} Mat[blk][d] u_{nbr_d(blk)} for
// the blocks at the listed owned positions (list null: positions 0..nlist-1).
// Mat is stored transposed, Mat[blk][d][l][k] = (block d of blk)[k][l], so
// the threads of a block's rows k read Mat coalesced in k (the vector entry
// u_{nbr_d}[l] is the same address for all of them). A thread sums all
// terms of one row (or, when the rows do not fill the workgroup, those of a
// contiguous range of d, the ranges meeting in lds in a fixed order), with
// kApplyChunk matrix and vector loads of kApplyD neighbour blocks in flight
// at a time, and writes its row without waiting for the others: y may alias
// u where the rows written and the entries read lie on different blocks (the
// even-odd updates). Ends with a workgroup barrier.
constexpr int kApplyChunk = 8;
template <typename T>
__device__ inline void apply_blocks(const LittleCtx<T>& c, const int* list, int nlist, const cpx<T>* __restrict__ Mat,
                                    int d0, int d1, const cpx<T>* u, const cpx<T>* s, double alpha, double beta,
                                    cpx<T>* y, double* lds)
{
    constexpr int kApplyD = 2;
    const Geom& g = c.a.g;
    const int Ns = c.a.Ns;
    const int nd = d1 - d0;
    const int rows = nlist * Ns;
    const int ng = rows > 0 ? max(1, min(LT1 / rows, nd)) : 1;
    const int per = (nd + ng - 1) / ng;
    for (int t0 = 0; t0 < ng * rows; t0 += LT1) {
        const int task = t0 + c.t;
        if (task < ng * rows) {
            const int gq = task / rows, row = task - gq * rows;
            const int ib = row / Ns, k = row - ib * Ns;
            const int own = list ? list[ib] : ib;
            const int blk = c.g + own * c.G;
            const int da = d0 + gq * per, dz = min(d1, da + per);
            double re = 0.0, im = 0.0;
            for (int db = da; db < dz; db += kApplyD) {
                const cpx<T>* M[kApplyD];
                const cpx<T>* uu[kApplyD];
#pragma unroll
                for (int v = 0; v < kApplyD; ++v) {
                    const int d = min(db + v, dz - 1);  // past dz: a valid block, dropped below
                    const int nb = d == 0 ? blk : (c.nbr ? c.nbr[8 * own + d - 1] : nbr_block(g, blk, d));
                    M[v] = Mat + ((long)blk * 9 + d) * Ns * Ns + k;
                    uu[v] = u + (long)nb * Ns;
                }
                for (int l0 = 0; l0 < Ns; l0 += kApplyChunk) {
                    cpx<T> mv[kApplyD][kApplyChunk], uv[kApplyD][kApplyChunk];
#pragma unroll
                    for (int v = 0; v < kApplyD; ++v)
#pragma unroll
                        for (int q = 0; q < kApplyChunk; ++q) {
                            const int l = min(l0 + q, Ns - 1);  // past Ns: re-read, dropped below
                            mv[v][q] = M[v][(long)l * Ns];
                            uv[v][q] = uu[v][l];
                        }
#pragma unroll
                    for (int v = 0; v < kApplyD; ++v)
#pragma unroll
                        for (int q = 0; q < kApplyChunk; ++q)
                            if (db + v < dz && l0 + q < Ns) {
                                const cpx<T> p = mv[v][q], w = uv[v][q];
                                re += (double)p.re * (double)w.re - (double)p.im * (double)w.im;
                                im += (double)p.re * (double)w.im + (double)p.im * (double)w.re;
                            }
                }
            }
            if (ng == 1) {
                const long i = (long)blk * Ns + k;
                double yr = beta * re, yi = beta * im;
                if (alpha != 0.0) {
                    yr += alpha * (double)s[i].re;
                    yi += alpha * (double)s[i].im;
                }
                y[i] = cpx<T>{(T)yr, (T)yi};
            } else {
                lds[2 * task] = re;
                lds[2 * task + 1] = im;
            }
        }
    }
    if (ng > 1) {
        __syncthreads();
        for (int row = c.t; row < rows; row += LT1) {
            double sr = 0.0, si = 0.0;
            for (int gq = 0; gq < ng; ++gq) {
                sr += lds[2 * (gq * rows + row)];
                si += lds[2 * (gq * rows + row) + 1];
            }
            const int ib = row / Ns, k = row - ib * Ns;
            const int blk = c.g + (list ? list[ib] : ib) * c.G;
            const long i = (long)blk * Ns + k;
            double yr = beta * sr, yi = beta * si;
            if (alpha != 0.0) {
                yr += alpha * (double)s[i].re;
                yi += alpha * (double)s[i].im;
            }
            y[i] = cpx<T>{(T)yr, (T)yi};
        }
    }
    __syncthreads();
}

// ||v||^2 over the workgroup's vector entries -> part[slot][g]
template <typename T>
__device__ inline void partial_norm2(const LittleCtx<T>& c, const cpx<T>* __restrict__ v, int slot, double* sh)
{
    double s = 0.0;
    const int R = c.R();
    for (int e = c.t; e < R; e += LT1) {
        cpx<T> z = v[c.entry(e)];
        s += (double)z.re * (double)z.re + (double)z.im * (double)z.im;
    }
    s = block_sum(s, sh);
    if (c.t == 0) {
        c.a.part[((long)slot * c.G + c.g) * 2] = s;
        c.a.part[((long)slot * c.G + c.g) * 2 + 1] = 0.0;
    }
}

// Partial sums of one Gram-Schmidt pass over the vector entries, one
// wavefront per slot: (chi_j, y) and (chi_j, r) for j < k, ||y||^2, (y, r)
// and (Q_l, y) for the nq global deflation directions, written to
// part[slot0 ...][g].
template <typename T>
__device__ inline void partial_pass(const LittleCtx<T>& c, const cpx<T>* chi, int k, const cpx<T>* __restrict__ y,
                                    const cpx<T>* __restrict__ r, int slot0, int nqg)
{
    constexpr int NW = LT1 / 64;
    const int lane = c.t & 63, w = c.t >> 6;
    const int ns = 2 * k + 2 + nqg;
    const int R = c.R();
    // kSlotUnroll slots per wavefront at a time, their loads in flight together
    for (int sb = w; sb < ns; sb += NW * kSlotUnroll) {
        double2 acc[kSlotUnroll];
        const cpx<T>* p[kSlotUnroll];
        const cpx<T>* q[kSlotUnroll];
#pragma unroll
        for (int u = 0; u < kSlotUnroll; ++u) {
            acc[u] = make_double2(0.0, 0.0);
            const int s = sb + u * NW;  // slots past ns read y (result dropped)
            if (s < k) {
                p[u] = chi + (long)s * c.N;
                q[u] = y;
            } else if (s < 2 * k) {
                p[u] = chi + (long)(s - k) * c.N;
                q[u] = r;
            } else if (s < 2 * k + 2) {
                p[u] = y;
                q[u] = (s == 2 * k) ? y : r;
            } else if (s < ns) {
                p[u] = c.a.Q + (long)(s - 2 * k - 2) * c.N;
                q[u] = y;
            } else {
                p[u] = y;
                q[u] = y;
            }
        }
        for (int e = lane; e < R; e += 64) {
            const long i = c.entry(e);
            cpx<T> pv[kSlotUnroll], qv[kSlotUnroll];
#pragma unroll
            for (int u = 0; u < kSlotUnroll; ++u) {
                pv[u] = p[u][i];
                qv[u] = q[u][i];
            }
#pragma unroll
            for (int u = 0; u < kSlotUnroll; ++u)
                acc[u] = cfma_conj(acc[u], (double)pv[u].re, (double)pv[u].im, (double)qv[u].re, (double)qv[u].im);
        }
#pragma unroll
        for (int u = 0; u < kSlotUnroll; ++u) {
            const int s = sb + u * NW;
            const double sr = wave_sum(acc[u].x), si = wave_sum(acc[u].y);
            if (s < ns && lane == 0) {
                c.a.part[((long)(slot0 + s) * c.G + c.g) * 2] = sr;
                c.a.part[((long)(slot0 + s) * c.G + c.g) * 2 + 1] = si;
            }
        }
    }
}

// ||v||^2 into slot sn and (Q_l, v), l < nq, into slots SQ + l (one wavefront per slot)
template <typename T>
__device__ inline void partial_norm2_q(const LittleCtx<T>& c, const cpx<T>* __restrict__ v, int sn)
{
    const int lane = c.t & 63, w = c.t >> 6;
    const int R = c.R();
    // minimal-residual form: (Q_l, v); oblique form: (Z_l, v) and (W_l, v)
    const int nd = c.a.oblique ? 2 * c.a.nq : c.a.nq;
    for (int s = w; s < 1 + nd; s += LT1 / 64) {
        const cpx<T>* u = s == 0 ? v
                          : (c.a.oblique && s <= c.a.nq) ? c.a.Z + (long)(s - 1) * c.N
                                                          : c.a.Q + (long)((s - 1) % c.a.nq) * c.N;
        double2 acc = make_double2(0.0, 0.0);
        for (int e = lane; e < R; e += 64) {
            long i = c.entry(e);
            cpx<T> p = u[i], q = v[i];
            acc = cfma_conj(acc, (double)p.re, (double)p.im, (double)q.re, (double)q.im);
        }
        acc.x = wave_sum(acc.x);
        acc.y = wave_sum(acc.y);
        if (lane == 0) {
            const int slot = s == 0 ? sn : SQ + s - 1;  // (W_l, v) follow the nq (Z_l, v)
            c.a.part[((long)slot * c.G + c.g) * 2] = acc.x;
            c.a.part[((long)slot * c.G + c.g) * 2 + 1] = acc.y;
        }
    }
}

// (Z_l, y), l < nq, into slots SQ + l (oblique deflation of a new Krylov image)
template <typename T>
__device__ inline void partial_zdots(const LittleCtx<T>& c, const cpx<T>* __restrict__ y)
{
    const int lane = c.t & 63, w = c.t >> 6;
    const int R = c.R();
    for (int s = w; s < c.a.nq; s += LT1 / 64) {
        const cpx<T>* u = c.a.Z + (long)s * c.N;
        double2 acc = make_double2(0.0, 0.0);
        for (int e = lane; e < R; e += 64) {
            long i = c.entry(e);
            cpx<T> p = u[i], q = y[i];
            acc = cfma_conj(acc, (double)p.re, (double)p.im, (double)q.re, (double)q.im);
        }
        acc.x = wave_sum(acc.x);
        acc.y = wave_sum(acc.y);
        if (lane == 0) {
            c.a.part[((long)(SQ + s) * c.G + c.g) * 2] = acc.x;
            c.a.part[((long)(SQ + s) * c.G + c.g) * 2 + 1] = acc.y;
        }
    }
}

// For each of the workgroup's entries e (entry index i): out(e, i, sr, si)
// with sr + i si = sum_{j < nterm} cf(j) v(j)[i], cf(j) a complex coefficient
// (double2) and v(j) a little vector. When the workgroup has few entries the
// terms of an entry are split over thread groups whose partial sums meet in
// lds (2 LT1 doubles, summed in a fixed order); loads are issued four terms
// at a time. Ends with a workgroup barrier.
constexpr int kTermChunk = 4;
template <typename T, typename CF, typename VF, typename OUT>
__device__ inline void combine_terms(const LittleCtx<T>& c, int nterm, CF cf, VF vf, double* lds, OUT out)
{
    const int R = c.R();
    const int ng = R > 0 ? max(1, min(LT1 / R, (nterm + kTermChunk - 1) / kTermChunk)) : 1;
    const int per = (nterm + ng - 1) / ng;
    for (int t = c.t; t < ng * R; t += LT1) {
        const int gq = t / R, e = t - gq * R;
        const long i = c.entry(e);
        double sr = 0.0, si = 0.0;
        const int ja = gq * per, jz = min(nterm, ja + per);
        for (int jb = ja; jb < jz; jb += kTermChunk) {
            cpx<T> zv[kTermChunk];
            double2 cv[kTermChunk];
#pragma unroll
            for (int u = 0; u < kTermChunk; ++u) {
                const int j = min(jb + u, jz - 1);  // past jz: a valid term with coefficient 0
                cv[u] = jb + u < jz ? cf(j) : make_double2(0.0, 0.0);
                zv[u] = vf(j)[i];
            }
#pragma unroll
            for (int u = 0; u < kTermChunk; ++u) {
                sr += cv[u].x * (double)zv[u].re - cv[u].y * (double)zv[u].im;
                si += cv[u].x * (double)zv[u].im + cv[u].y * (double)zv[u].re;
            }
        }
        if (ng > 1) {
            lds[2 * t] = sr;
            lds[2 * t + 1] = si;
        } else {
            out(e, i, sr, si);
        }
    }
    if (ng > 1) {
        __syncthreads();
        for (int e = c.t; e < R; e += LT1) {
            double sr = 0.0, si = 0.0;
            for (int gq = 0; gq < ng; ++gq) {
                sr += lds[2 * (gq * R + e)];
                si += lds[2 * (gq * R + e) + 1];
            }
            out(e, c.entry(e), sr, si);
        }
    }
    __syncthreads();
}

// GCR on A v = w (EO = false) or on the even-odd reduced system (EO = true,
// appendix A.2): with D the block diagonal of A and M_d = D^-1 A_d,
//   v_e solves (1 - M_eo M_oe) v_e = (D^-1 w)_e - M_eo (D^-1 w)_o,
//   v_o = (D^-1 w)_o - M_oe v_e.
// Even-odd workspaces: w1 = D^-1 w (all blocks); w2 holds the reduced source
// on even blocks and the intermediate M_oe u on odd blocks.
template <typename T, bool EO> __global__ __launch_bounds__(LT1) void k_little_gcr(LittleArgs<T> a)
{
    // FP64: the residue norm inside a cycle follows from the coefficients
    // while it is more than kNormFloor ||w||^2 above the tolerance
    constexpr bool kTrackNorm = sizeof(T) == sizeof(double);
    constexpr double kNormFloor = 1e-12;
    // FP64 solves to a relative tolerance of 1e-8 or looser end on the
    // measured recursive residue (its drift from the true one is ~1e-15);
    // tighter ones, and FP32 solves, confirm it by recomputing w - A x
    constexpr double kLooseTol2 = 1e-16;
    __shared__ double red[2 * (2 * NK + 2 + NQ)];
    __shared__ double acoef[NK][NK][2];
    __shared__ double qcoef[NQ][NK][2];  // components of each direction's image along Q
    __shared__ double zc[NQ][2];
    __shared__ double cq_s[NQ][2];       // coefficients of the current projection along W (or Q) and Z
    __shared__ double pn2_s;             // ||r||^2 after a projection
    __shared__ double bcoef[NK];
    __shared__ double ccoef[NK][2];
    __shared__ double alpha[NK][2];
    __shared__ double sh[16];
    __shared__ double wn2_s, rn2_s;
    __shared__ int second_s;
    __shared__ int last_s;
    __shared__ double lds[2 * LT1];
    __shared__ int l_even[EO ? kMaxOwned : 1], l_odd[EO ? kMaxOwned : 1];  // owned positions by colour
    __shared__ int n_even_s, n_odd_s;
    __shared__ int nbr_tab[8 * kMaxOwned];  // neighbours of the owned blocks, computed once

    const int G = (int)gridDim.x, gi = (int)blockIdx.x, t = (int)threadIdx.x;
    const int nbg = (a.g.Nb - gi + G - 1) / G;
    const bool tab = nbg <= kMaxOwned;
    if (tab)
        for (int q = t; q < 8 * nbg; q += LT1)
            nbr_tab[q] = nbr_block(a.g, gi + (q >> 3) * G, 1 + (q & 7));
    if (EO && t == 0) {
        int ne = 0, no = 0;
        for (int i = 0; i < nbg; ++i) {
            if (block_colour(a.g, gi + i * G))
                l_odd[no++] = i;
            else
                l_even[ne++] = i;
        }
        n_even_s = ne;
        n_odd_s = no;
    }
    __syncthreads();
    const int n_even = EO ? n_even_s : 0, n_odd = EO ? n_odd_s : 0;
    LittleCtx<T> c{a, G, gi, t, (long)a.g.Nb * a.Ns, EO ? l_even : nullptr, EO ? n_even : nbg, tab ? nbr_tab : nullptr};
    const double tol2 = a.tol_dev ? (*a.tol_dev) * (*a.tol_dev) : a.tol2;
    unsigned long long bar_target = 0;
    if (c.t == 0)
        bar_target = __hip_atomic_load(a.bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const long N = c.N;
    const int R = c.R();
    // op: y = A u (plain) or y = u - M_eo M_oe u on even blocks (one more barrier)
    auto op = [&](const cpx<T>* u, cpx<T>* y) {
        if (EO) {
            apply_blocks(c, l_odd, n_odd, a.Mt, 1, 9, u, (const cpx<T>*)nullptr, 0.0, 1.0, a.w2, lds);
            grid_barrier(a.bar_count, a.bar_gen, bar_target, a.stats);
            apply_blocks(c, l_even, n_even, a.Mt, 1, 9, (const cpx<T>*)a.w2, u, 1.0, -1.0, y, lds);
        } else {
            apply_blocks(c, (const int*)nullptr, nbg, a.At, 0, 9, u, (const cpx<T>*)nullptr, 0.0, 1.0, y, lds);
        }
    };
    // a grid barrier whose last arrival reduces slots [s0, s0 + ns) into red for everyone
    double* const pub = a.part + (long)NSLOT * G * 2;
    auto barrier_reduce = [&](int s0, int ns) {
        grid_barrier_reduce(a.bar_count, a.bar_gen, bar_target, a.stats, a.part, pub, G, s0, ns, red, &last_s);
    };
    // red[q] = red[from + q], q < n (then a workgroup barrier)
    auto shift_red = [&](int from, int n) {
        const double v = c.t < n ? red[from + c.t] : 0.0;
        __syncthreads();
        if (c.t < n)
            red[c.t] = v;
        __syncthreads();
    };
    const cpx<T>* rhs = a.w;
    if (EO) {
        apply_blocks(c, (const int*)nullptr, nbg, a.Mt, 0, 1, a.w, (const cpx<T>*)nullptr, 0.0, 1.0, a.w1, lds);
        grid_barrier(a.bar_count, a.bar_gen, bar_target, a.stats);
        apply_blocks(c, l_even, n_even, a.Mt, 1, 9, (const cpx<T>*)a.w1, (const cpx<T>*)a.w1, 1.0, -1.0, a.w2, lds);
        rhs = a.w2;
    }

    const int nq = a.nq;
    const bool obl = a.oblique && nq > 0;
    const int nqg = obl ? 0 : nq;  // deflation directions inside the Gram-Schmidt pass (minimal-residual form)
    // Coefficients of the projection of a vector v whose dots sit in red
    // ((Q_l, v) or (Z_l, v) at 0.., (W_l, v) at 2 nq.. in the oblique form):
    // c = (Q_l, v) (Q orthonormal), or c = Ainv Z^+ v (section 3's P_L on the
    // even-odd system, Ainv the inverse of the little little operator Z^+ A_hat Z).
    // Returns ||v - Q c||^2 given ||v||^2 (thread 0's value is authoritative).
    auto proj_coef = [&](double vn2) {
        if (c.t < nq) {
            double cr = red[2 * c.t], ci = red[2 * c.t + 1];
            if (obl) {
                cr = 0.0;
                ci = 0.0;
                for (int m = 0; m < nq; ++m) {
                    const double ar = a.Ainv[2 * (c.t * nq + m)], ai = a.Ainv[2 * (c.t * nq + m) + 1];
                    cr += ar * red[2 * m] - ai * red[2 * m + 1];
                    ci += ar * red[2 * m + 1] + ai * red[2 * m];
                }
            }
            cq_s[c.t][0] = cr;
            cq_s[c.t][1] = ci;
        }
        __syncthreads();
        double rn = vn2;
        if (c.t == 0) {
            if (!obl) {
                for (int l = 0; l < nq; ++l)
                    rn -= cq_s[l][0] * cq_s[l][0] + cq_s[l][1] * cq_s[l][1];
            } else {
                // ||v - W c||^2 = ||v||^2 - 2 Re sum conj(c_l) (W_l, v) + c^+ Gw c
                for (int l = 0; l < nq; ++l) {
                    const double cr = cq_s[l][0], ci = cq_s[l][1];
                    const double wr = red[2 * (nq + l)], wi = red[2 * (nq + l) + 1];
                    rn -= 2.0 * (cr * wr + ci * wi);
                    for (int m = 0; m < nq; ++m) {
                        const double gr = a.Gw[2 * (l * nq + m)], gi = a.Gw[2 * (l * nq + m) + 1];
                        const double dr = cq_s[m][0], di = cq_s[m][1];
                        // conj(c_l) G_lm c_m
                        const double tr = gr * dr - gi * di, ti = gr * di + gi * dr;
                        rn += cr * tr + ci * ti;
                    }
                }
            }
        }
        return rn;
    };
    // r -= Q c (or W c), x += Z c with c = cq_s: the residue leaves span Q (minimal-residual
    // form) or range(A_hat Z) along the oblique projector (section 3)
    auto project_q = [&]() {
        auto cq = [&](int l) { return make_double2(cq_s[l][0], cq_s[l][1]); };
        combine_terms(c, nq, cq, [&](int l) { return a.Q + (long)l * N; }, lds, [&](int, long i, double sr, double si) {
            a.r[i] = cpx<T>{(T)((double)a.r[i].re - sr), (T)((double)a.r[i].im - si)};
        });
        combine_terms(c, nq, cq, [&](int l) { return a.Z + (long)l * N; }, lds, [&](int, long i, double sr, double si) {
            a.x[i] = cpx<T>{(T)((double)a.x[i].re + sr), (T)((double)a.x[i].im + si)};
        });
    };

    // x = 0, r = rhs, ||rhs||^2 and (Q, rhs); then r leaves span Q
    for (int e = c.t; e < R; e += LT1) {
        long i = c.entry(e);
        a.x[i] = cpx<T>{0, 0};
        a.r[i] = rhs[i];
    }
    partial_norm2_q(c, rhs, SW);
    // SW and the SQ slots are adjacent: one reduction, then the (Q_l, rhs) moved to red[0..]
    const int nqd = nq > 0 ? (obl ? 2 * nq : nq) : 0;
    barrier_reduce(SW, 1 + nqd);
    if (c.t == 0)
        wn2_s = red[0];
    shift_red(2, 2 * nqd);
    const double wn2 = wn2_s;
    double rn2_0 = wn2;  // ||r||^2 after the projection below (thread 0)
    if (nq > 0) {
        rn2_0 = proj_coef(wn2);
        project_q();
    }
    if (c.t == 0)
        rn2_s = rn2_0;
    __syncthreads();
    int iters = 0;
    bool converged = !(wn2 > 0.0);
    bool broke = false;
    bool hit = false;      // the last cycle ended on the measured ||r||^2 <= tol^2 ||w||^2
    bool skipped = false;  // ... and the solve ended there without recomputing the residue

    // Every branch below depends only on values reduced identically by all
    // workgroups, so all of them pass the same sequence of grid barriers.
    while (!converged && !broke && iters < a.maxiter) {
        int k = 0;
        hit = false;
        for (; k < a.nkv && iters < a.maxiter; ++k) {
            cpx<T>* xk = a.xi + (long)k * N;
            cpx<T>* ck = a.chi + (long)k * N;
            cpx<T>* xnext = a.xi + (long)(k + 1) * N;  // used only while k + 1 < nkv
            // ||r||^2 inside a cycle: in FP64 it follows from the coefficients
            // (||r_k||^2 = ||r_{k-1}||^2 - |c_k|^2, chi_k a unit vector
            // orthogonal to r_k), but that difference carries an absolute
            // error of a few ulp of ||w||^2. While the estimate lies well
            // above the tolerance it only says "not converged" and the
            // reduction is skipped; near the tolerance, and always in single
            // precision, ||r||^2 is measured. The true residue is recomputed
            // and tested at every restart.
            const bool far = k > 0 && kTrackNorm && rn2_s > (tol2 + kNormFloor) * wn2;
            if (k == 0 || far) {
                if (k == 0)
                    for (int e = c.t; e < R; e += LT1) {
                        long i = c.entry(e);
                        xk[i] = a.r[i];  // xi_k = r (else written by the previous step's update)
                    }
                grid_barrier(a.bar_count, a.bar_gen, bar_target, a.stats);  // S1: xi_k complete everywhere
            } else {
                for (int e = c.t; e < R; e += LT1) {
                    long i = c.entry(e);
                    xk[i] = a.r[i];
                }
                partial_norm2(c, a.r, SC, sh);
                barrier_reduce(SC, 1);  // S1: r complete everywhere
                if (c.t == 0)
                    rn2_s = red[0];
                __syncthreads();
                if (rn2_s <= tol2 * wn2) {
                    hit = true;
                    break;  // converged with k directions
                }
            }
            op(xk, ck);
            if (obl) {
                // oblique form: chi_k = P_L A_hat xi_k = A_hat xi_k - W Ainv Z^+ A_hat xi_k
                // before the Gram-Schmidt pass (one more reduction); the
                // preimage of chi_k is xi_k - Z c_k
                __syncthreads();
                partial_zdots(c, ck);
                barrier_reduce(SQ, nq);
                proj_coef(0.0);
                if (c.t < nq) {
                    qcoef[c.t][k][0] = cq_s[c.t][0];
                    qcoef[c.t][k][1] = cq_s[c.t][1];
                }
                combine_terms(c, nq, [&](int l) { return make_double2(cq_s[l][0], cq_s[l][1]); },
                              [&](int l) { return a.Q + (long)l * N; }, lds, [&](int, long i, double sr, double si) {
                                  ck[i] = cpx<T>{(T)((double)ck[i].re - sr), (T)((double)ck[i].im - si)};
                              });
            }
            // one Gram-Schmidt pass: everything needed for chi_k, c_k and the new r
            partial_pass(c, a.chi, k, ck, a.r, SA, nqg);
            barrier_reduce(SA, 2 * k + 2 + nqg);  // S2
            // red: [0,k) a_j; [k,2k) (chi_j, r); 2k: ||chi_k||^2; 2k+1: (chi_k, r); [2k+2, 2k+2+nq) (Q_l, chi_k)
            const int q0 = 2 * k + 2;
            // the k + nq <= 64 projections are spread over the lanes of wavefront 0
            if (c.t < 64) {
                const int ri = c.t < k ? 2 * c.t : 2 * (q0 + c.t - k);
                const double m2 = c.t < k + nqg ? red[ri] * red[ri] + red[ri + 1] * red[ri + 1] : 0.0;
                const double p2 = wave_sum(m2);
                if (c.t == 0) {
                    const double n2 = red[4 * k];
                    second_s = ((k > 0 || nqg > 0) && !(n2 - p2 >= 0.01 * n2)) ? 1 : 0;
                }
            }
            __syncthreads();
            if (second_s) {
                // heavy cancellation: subtract the first projections, then a second pass
                for (int e = c.t; e < R; e += LT1) {
                    long i = c.entry(e);
                    double yr = (double)ck[i].re, yi = (double)ck[i].im;
#pragma unroll 8
                    for (int j = 0; j < k; ++j) {
                        cpx<T> z = a.chi[(long)j * N + i];
                        yr -= red[2 * j] * (double)z.re - red[2 * j + 1] * (double)z.im;
                        yi -= red[2 * j] * (double)z.im + red[2 * j + 1] * (double)z.re;
                    }
                    for (int l = 0; l < nqg; ++l) {
                        const double qr = red[2 * (q0 + l)], qi = red[2 * (q0 + l) + 1];
                        const cpx<T> z = a.Q[(long)l * N + i];
                        yr -= qr * (double)z.re - qi * (double)z.im;
                        yi -= qr * (double)z.im + qi * (double)z.re;
                    }
                    ck[i] = cpx<T>{(T)yr, (T)yi};
                }
                if (c.t < k) {
                    acoef[c.t][k][0] = red[2 * c.t];
                    acoef[c.t][k][1] = red[2 * c.t + 1];
                }
                if (c.t < nqg) {
                    qcoef[c.t][k][0] = red[2 * (q0 + c.t)];
                    qcoef[c.t][k][1] = red[2 * (q0 + c.t) + 1];
                }
                __syncthreads();
                partial_pass(c, a.chi, k, ck, a.r, SB, nqg);
                barrier_reduce(SB, 2 * k + 2 + nqg);  // S3
            } else {
                if (c.t < k) {
                    acoef[c.t][k][0] = 0.0;
                    acoef[c.t][k][1] = 0.0;
                }
                if (c.t < nqg) {
                    qcoef[c.t][k][0] = 0.0;
                    qcoef[c.t][k][1] = 0.0;
                }
            }
            // red now holds the (last) pass: a_j, (chi_j, r), ||chi||^2, (chi, r)
            if (c.t < 64) {
                // lane j < k: chi_j; lane k + l: Q_l
                double m2 = 0.0, dr = 0.0, di = 0.0;
                if (c.t < k) {
                    const int j = c.t;
                    const double ar = red[2 * j], ai = red[2 * j + 1];
                    const double qr = red[2 * (k + j)], qi = red[2 * (k + j) + 1];
                    m2 = ar * ar + ai * ai;
                    // (chi - sum a_j chi_j, r) = (chi, r) - sum conj(a_j) (chi_j, r)
                    dr = ar * qr + ai * qi;
                    di = ar * qi - ai * qr;
                    acoef[j][k][0] += ar;
                    acoef[j][k][1] += ai;
                } else if (c.t < k + nqg) {
                    const int l = c.t - k;
                    const double qr = red[2 * (q0 + l)], qi = red[2 * (q0 + l) + 1];
                    m2 = qr * qr + qi * qi;
                    qcoef[l][k][0] += qr;
                    qcoef[l][k][1] += qi;
                }
                m2 = wave_sum(m2);
                dr = wave_sum(dr);
                di = wave_sum(di);
                if (c.t == 0) {
                    const double b2 = red[4 * k] - m2;
                    const double crr = red[4 * k + 2] - dr, cri = red[4 * k + 3] - di;
                    const double b = b2 > 0.0 ? sqrt(b2) : 0.0;
                    bcoef[k] = b;
                    ccoef[k][0] = b > 0.0 ? crr / b : 0.0;
                    ccoef[k][1] = b > 0.0 ? cri / b : 0.0;
                    if (kTrackNorm)
                        rn2_s -= ccoef[k][0] * ccoef[k][0] + ccoef[k][1] * ccoef[k][1];
                }
            }
            __syncthreads();
            const double b = bcoef[k];
            if (!(b > 0.0)) {
                broke = true;  // the new direction lies in the span: end the cycle without it
                break;
            }
            const double inv = 1.0 / b, cr0 = ccoef[k][0], ci0 = ccoef[k][1];
            // chi_k -= sum_j a_j chi_j + sum_l q_l Q_l, then normalise; r -= c_k chi_k
            combine_terms(
                c, k + nqg,
                [&](int j) {
                    const int ri = j < k ? 2 * j : 2 * (q0 + j - k);
                    return make_double2(red[ri], red[ri + 1]);
                },
                [&](int j) { return j < k ? a.chi + (long)j * N : a.Q + (long)(j - k) * N; }, lds,
                [&](int, long i, double sr, double si) {
                    double yr = ((double)ck[i].re - sr) * inv, yi = ((double)ck[i].im - si) * inv;
                    ck[i] = cpx<T>{(T)yr, (T)yi};
                    double rr = (double)a.r[i].re - (cr0 * yr - ci0 * yi);
                    double ri = (double)a.r[i].im - (cr0 * yi + ci0 * yr);
                    a.r[i] = cpx<T>{(T)rr, (T)ri};
                    if (kTrackNorm && k + 1 < a.nkv)
                        xnext[i] = cpx<T>{(T)rr, (T)ri};  // xi_{k+1} = r
                });
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
        // the direction preimages are xi_k - Z q_k: zc = sum_k q_k alpha_k
        if (c.t < nq) {
            double zr = 0.0, zi = 0.0;
            for (int j = 0; j < k; ++j) {
                zr += qcoef[c.t][j][0] * alpha[j][0] - qcoef[c.t][j][1] * alpha[j][1];
                zi += qcoef[c.t][j][0] * alpha[j][1] + qcoef[c.t][j][1] * alpha[j][0];
            }
            zc[c.t][0] = zr;
            zc[c.t][1] = zi;
        }
        __syncthreads();
        // x += sum_j alpha_j xi_j - sum_l zc_l Z_l
        combine_terms(
            c, k + nq,
            [&](int j) {
                return j < k ? make_double2(alpha[j][0], alpha[j][1]) : make_double2(-zc[j - k][0], -zc[j - k][1]);
            },
            [&](int j) { return j < k ? a.xi + (long)j * N : a.Z + (long)(j - k) * N; }, lds,
            [&](int, long i, double sr, double si) {
                a.x[i] = cpx<T>{(T)((double)a.x[i].re + sr), (T)((double)a.x[i].im + si)};
            });
        if (kTrackNorm && hit && tol2 >= kLooseTol2) {
            converged = true;
            skipped = true;
            break;
        }
        // recompute r = rhs - op(x)
        grid_barrier(a.bar_count, a.bar_gen, bar_target, a.stats);
        op(a.x, a.r);
        __syncthreads();
        for (int e = c.t; e < R; e += LT1) {
            long i = c.entry(e);
            a.r[i] = cpx<T>{(T)((double)rhs[i].re - (double)a.r[i].re), (T)((double)rhs[i].im - (double)a.r[i].im)};
        }
        // partial_norm2_q reads each entry from another thread than the one that wrote it
        __syncthreads();
        partial_norm2_q(c, a.r, SR);
        // slots SR, SW (not used here) and SQ.. in one reduction; the (Q_l, r) then moved to red[0..]
        barrier_reduce(SR, 2 + nqd);
        if (c.t == 0)
            rn2_s = red[0];
        shift_red(4, 2 * nqd);
        double rn2 = rn2_s;
        if (nq > 0) {
            // project the residue (x moves along Z); ||r||^2 as it is afterwards
            rn2 = proj_coef(rn2);
            if (c.t == 0)
                pn2_s = rn2;  // thread 0's value, shared below
            project_q();
            __syncthreads();
            rn2 = pn2_s;
        }
        converged = rn2 <= tol2 * wn2;
        __syncthreads();  // every thread has read rn2_s
        if (c.t == 0)
            rn2_s = rn2;  // start of the next cycle's norm updates
        __syncthreads();
    }
    if (EO) {
        // x_e must be complete everywhere: a barrier followed its last GCR
        // update unless the solve ended without the residue recomputation,
        // and none followed the projection along Z that may come after it
        if (nq > 0 || skipped)
            grid_barrier(a.bar_count, a.bar_gen, bar_target, a.stats);
        apply_blocks(c, l_odd, n_odd, a.Mt, 1, 9, (const cpx<T>*)a.x, (const cpx<T>*)a.w1, 1.0, -1.0, a.x, lds);
    }
    if (c.g == 0 && c.t == 0) {
        atomicAdd(&a.stats[0], iters);
        atomicAdd(&a.stats[1], 1);
        if (!converged)
            atomicOr(&a.stats[2], 1);
    }
}

// ------------------------------------------------------------ many sources
//
// The same GCR for nrhs little systems A v_b = w_b at once: the right-hand
// sides share the launch, the grid barriers and the reads of A, and each has
// its own Krylov space, coefficients and convergence test. Vectors of RHS b
// sit at b * N (w, x, r) and at (k * nrhs + b) * N (xi_k, chi_k).
// Reductions over the workgroups are two-level: partial sums, a barrier,
// workgroup g sums the slots t = g mod G into fin, a barrier, everyone reads
// fin. A RHS leaves the cycle when it converges or its new direction falls
// in the span; the cycle ends when no RHS is left in it. With EO the systems
// are the even-odd reduced ones of appendix A.2, as in the single-source
// solver: the Krylov vectors live on the even blocks, w1 = M_0 w holds each
// source's block-diagonally scaled right-hand side, w2 the reduced one on the
// even blocks and the operator's intermediate on the odd ones, and the odd
// part of each solution follows from the even part at the end.

constexpr int RS = 2 * NK + 2;  // slots of one pass per RHS

template <typename T> struct LittleMultiArgs {
    Geom g;
    int Ns, nkv, maxiter, nrhs;
    double tol2;
    const double* tol_dev;
    const cpx<T>* At;
    const cpx<T>* Mt;  // even-odd matrices (even-odd kernel only)
    cpx<T>* w1;        // M_0 w, nrhs vectors (even-odd kernel only)
    cpx<T>* w2;        // the reduced right-hand sides on even blocks, the odd-block intermediate of the operator
    const cpx<T>* w;
    cpx<T>* x;
    cpx<T>* r;
    cpx<T>* xi;
    cpx<T>* chi;
    double* part;   // [NSLOT][nrhs][G] complex
    double* fin;    // [nrhs][RS] complex
    double* acoef;  // [G][nrhs][NK][NK] complex (each workgroup's own copy)
    int* stats;
    unsigned* bar_count;
    unsigned long long* bar_gen;
};

template <typename T> struct MultiCtx {
    const LittleMultiArgs<T>& a;
    int G, g, t, nbg, R;
    long N;
    const int* vb;  // positions of the blocks the vectors live on (even-odd: the even ones), null: all owned
    __device__ long entry(int e) const
    {
        int i = e / a.Ns;
        int k = e - i * a.Ns;
        return (long)(g + (vb ? vb[i] : i) * G) * a.Ns + k;
    }
    __device__ double* pslot(int slot, int b) const { return a.part + (((long)slot * a.nrhs + b) * G + g) * 2; }
};

// y_b = alpha s_b + beta sum_{d0 <= d < d1} M_d v_b on owned blocks for the
// listed sources, on the matrix cores: for an owned block the terms
// sum_d M_d V_d (V_d: the listed sources' entries on the d-th neighbour, Ns x
// nlist) form one real GEMM of the 2Ns x 2(d1-d0)Ns matrix [[ar, -ai], [ai, ar]]
// (rows and columns interleaved re/im) with the 2(d1-d0)Ns x nlist matrix of
// the V_d entries read as reals, in 16x16x4 tiles (FP32 or FP64 MFMA). Wave w
// takes (block, row tile) tasks w, w + 16, ...; the sources (<= 16) are the
// 16 columns. M (A or the even-odd matrices) is read from transposed blocks,
// coalesced in the row. pos lists the npos owned positions to apply on (null:
// positions 0..npos-1); s is read only when alpha is not zero.
template <typename T> struct Mfma;
// Operands: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]; result
// element i of lane l is D[row(l / 16, i)][l % 16], with the row order of
// the FP32 and FP64 instructions differing.
template <> struct Mfma<float> {
    using acc_t = __attribute__((ext_vector_type(4))) float;
    static __device__ inline acc_t step(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int kq, int i) { return 4 * kq + i; }
};
template <> struct Mfma<double> {
    using acc_t = __attribute__((ext_vector_type(4))) double;
    static __device__ inline acc_t step(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int kq, int i) { return 4 * i + kq; }
};

constexpr int kMfmaBatch = 6;  // MFMA steps whose operands are in flight together (2 Ns = 48: two batches)
template <typename T>
__device__ inline void apply_multi_mfma(const MultiCtx<T>& c, const cpx<T>* __restrict__ Mat, int d0, int d1,
                                        const int* pos, int npos, const cpx<T>* __restrict__ v, const cpx<T>* s,
                                        double alpha, double beta, cpx<T>* y, const int* list, int nlist)
{
    const Geom& g = c.a.g;
    const int Ns = c.a.Ns;
    const int mt = (2 * Ns + 15) / 16;
    const int lane = c.t & 63, wave = c.t >> 6;
    const int n = lane & 15, kq = lane >> 4;
    const int b_n = n < nlist ? list[n] : 0;
    for (int task = wave; task < npos * mt; task += LT / 64) {
        const int ib = task / mt, tt = task - ib * mt;
        const int blk = c.g + (pos ? pos[ib] : ib) * c.G;
        const int rr = 16 * tt + n;
        const int m = rr >> 1, cr = rr & 1;
        typename Mfma<T>::acc_t acc = {0, 0, 0, 0};
#pragma unroll 1
        for (int d = d0; d < d1; ++d) {
            const int nbr = nbr_block(g, blk, d);
            const cpx<T>* Ad = Mat + ((long)blk * 9 + d) * Ns * Ns;
            const cpx<T>* vb = v + b_n * c.N + (long)nbr * Ns;
            // the operands of kMfmaBatch steps loaded together, then their products
#pragma unroll 1
            for (int kc0 = 0; kc0 < 2 * Ns; kc0 += 4 * kMfmaBatch) {
                T av[kMfmaBatch], bw[kMfmaBatch];
                // clamped indices: every load is issued (no branch between them), the
                // out-of-range operands are zeroed afterwards
                cpx<T> za[kMfmaBatch], qa[kMfmaBatch];
#pragma unroll
                for (int st = 0; st < kMfmaBatch; ++st) {
                    const int kk = min(kc0 + 4 * st + kq, 2 * Ns - 1);
                    const int l = kk >> 1;
                    za[st] = Ad[(long)l * Ns + min(m, Ns - 1)];
                    qa[st] = vb[l];
                }
#pragma unroll
                for (int st = 0; st < kMfmaBatch; ++st) {
                    const int kk = kc0 + 4 * st + kq;
                    const int ck = kk & 1;
                    const bool in = kk < 2 * Ns;
                    const cpx<T> z = za[st], q = qa[st];
                    av[st] = (in && m < Ns) ? (cr == 0 ? (ck == 0 ? z.re : -z.im) : (ck == 0 ? z.im : z.re)) : T(0);
                    bw[st] = (in && n < nlist) ? (ck == 0 ? q.re : q.im) : T(0);
                }
#pragma unroll
                for (int st = 0; st < kMfmaBatch; ++st)
                    if (kc0 + 4 * st < 2 * Ns)
                        acc = Mfma<T>::step(av[st], bw[st], acc);
            }
        }
        if (n < nlist) {
            const long o = b_n * c.N + (long)blk * Ns;
            T* yb = reinterpret_cast<T*>(y + o);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ro = 16 * tt + Mfma<T>::row(kq, i);
                if (ro < 2 * Ns) {
                    double val = beta * (double)acc[i];
                    if (alpha != 0.0)
                        val += alpha * (double)reinterpret_cast<const T*>(s + o)[ro];
                    yb[ro] = (T)val;
                }
            }
        }
    }
    __syncthreads();
}

// part[slot][b][g] = ||v_b||^2 over the owned entries, one wavefront per listed RHS
template <typename T>
__device__ inline void multi_norm2(const MultiCtx<T>& c, const cpx<T>* v, const int* list, int nlist, int slot)
{
    const int lane = c.t & 63, wv = c.t >> 6;
    for (int bi = wv; bi < nlist; bi += LT / 64) {
        const int b = list[bi];
        const cpx<T>* vb = v + b * c.N;
        double s = 0.0;
        for (int e = lane; e < c.R; e += 64) {
            cpx<T> z = vb[c.entry(e)];
            s += (double)z.re * (double)z.re + (double)z.im * (double)z.im;
        }
        s = wave_sum(s);
        if (lane == 0) {
            double* p = c.pslot(slot, b);
            p[0] = s;
            p[1] = 0.0;
        }
    }
}

// every workgroup: out[b] = sum over workgroups of part[slot][b] (real part), listed RHS
__device__ inline void multi_reduce_real(const double* part, int nrhs, int G, int slot, const int* list, int nlist,
                                         double* out)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int bi = wv; bi < nlist; bi += LT / 64) {
        const int b = list[bi];
        double s = 0.0;
        for (int q = lane; q < G; q += 64)
            s += part[(((long)slot * nrhs + b) * G + q) * 2];
        s = wave_sum(s);
        if (lane == 0)
            out[b] = s;
    }
    __syncthreads();
}

// Gram-Schmidt partial sums for the listed RHS into slots slot0 + s, s < 2k+2
// (same layout as partial_pass). One wavefront per (RHS, group of 8 slots):
// the lanes run over the workgroup's entries, y and r are read once for the
// group, and the 8 complex sums are reduced across the wavefront at the end.
constexpr int kSlotGroup = 8;

template <typename T>
__device__ inline void multi_pass(const MultiCtx<T>& c, int k, const int* list, int nlist, int slot0)
{
    const int ns = 2 * k + 2;
    const int ngrp = (ns + kSlotGroup - 1) / kSlotGroup;
    const int lane = c.t & 63, wv = c.t >> 6;
    const long N = c.N;
    const int nr = c.a.nrhs;
    for (int task = wv; task < nlist * ngrp; task += LT / 64) {
        const int bi = task / ngrp, s0 = (task - bi * ngrp) * kSlotGroup;
        const int b = list[bi];
        const cpx<T>* y = c.a.chi + ((long)k * nr + b) * N;
        const cpx<T>* r = c.a.r + b * N;
        double2 acc[kSlotGroup];
#pragma unroll
        for (int q = 0; q < kSlotGroup; ++q)
            acc[q] = make_double2(0.0, 0.0);
        for (int e = lane; e < c.R; e += 64) {
            const long i = c.entry(e);
            const cpx<T> yv = y[i], rv = r[i];
#pragma unroll
            for (int q = 0; q < kSlotGroup; ++q) {
                const int sl = s0 + q;
                if (sl < ns) {
                    cpx<T> u, v;
                    if (sl < 2 * k) {
                        u = c.a.chi[((long)(sl < k ? sl : sl - k) * nr + b) * N + i];
                        v = sl < k ? yv : rv;
                    } else {
                        u = yv;
                        v = sl == 2 * k ? yv : rv;
                    }
                    acc[q] = cfma_conj(acc[q], (double)u.re, (double)u.im, (double)v.re, (double)v.im);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < kSlotGroup; ++q) {
            if (s0 + q >= ns)
                break;
            const double re = wave_sum(acc[q].x), im = wave_sum(acc[q].y);
            if (lane == 0) {
                double* p = c.pslot(slot0 + s0 + q, b);
                p[0] = re;
                p[1] = im;
            }
        }
    }
}

// workgroup g: fin[b][s] = sum over workgroups of part[slot0 + s][b], for the
// (listed RHS, s < ns) tasks t with t mod G == g
__device__ inline void multi_fin(const double* part, double* fin, int nrhs, int G, int g, int slot0, int ns,
                                 const int* list, int nlist)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ntask = nlist * ns;
    int j = 0;
    for (int task = g; task < ntask; task += G, ++j) {
        if ((j % (LT / 64)) != wv)
            continue;
        const int bi = task / ns, s = task - bi * ns;
        const int b = list[bi];
        double re = 0.0, im = 0.0;
        for (int q = lane; q < G; q += 64) {
            re += part[((((long)slot0 + s) * nrhs + b) * G + q) * 2];
            im += part[((((long)slot0 + s) * nrhs + b) * G + q) * 2 + 1];
        }
        re = wave_sum(re);
        im = wave_sum(im);
        if (lane == 0) {
            fin[((long)b * RS + s) * 2] = re;
            fin[((long)b * RS + s) * 2 + 1] = im;
        }
    }
}

template <typename T, bool EO> __global__ __launch_bounds__(LT) void k_little_gcr_multi(LittleMultiArgs<T> a)
{
    __shared__ double red[kMaxLittleRhs][2 * RS];
    __shared__ double bcoef[kMaxLittleRhs][NK];
    __shared__ double ccoef[kMaxLittleRhs][NK][2];
    __shared__ double alpha[kMaxLittleRhs][NK][2];
    __shared__ double wn2[kMaxLittleRhs], rn2[kMaxLittleRhs];
    __shared__ int act[kMaxLittleRhs], stop[kMaxLittleRhs], conv[kMaxLittleRhs], kb[kMaxLittleRhs];
    __shared__ int second[kMaxLittleRhs];
    __shared__ int list[kMaxLittleRhs], nlist_s, list2[kMaxLittleRhs], nlist2_s;
    __shared__ int l_even[EO ? kMaxOwned : 1], l_odd[EO ? kMaxOwned : 1];  // owned positions by colour
    __shared__ int n_even_s, n_odd_s;

    MultiCtx<T> c{a, (int)gridDim.x, (int)blockIdx.x, (int)threadIdx.x, 0, 0, (long)a.g.Nb * a.Ns, nullptr};
    const double tol2 = a.tol_dev ? (*a.tol_dev) * (*a.tol_dev) : a.tol2;
    const int nr = a.nrhs;
    const long N = c.N;
    unsigned long long bar_target = 0;
    if (c.t == 0)
        bar_target = __hip_atomic_load(a.bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    c.nbg = (a.g.Nb - c.g + c.G - 1) / c.G;
    if (EO && c.t == 0) {
        int ne = 0, no = 0;
        for (int i = 0; i < c.nbg; ++i) {
            if (block_colour(a.g, c.g + i * c.G))
                l_odd[no++] = i;
            else
                l_even[ne++] = i;
        }
        n_even_s = ne;
        n_odd_s = no;
    }
    if (c.t < nr)
        list[c.t] = c.t;
    if (c.t == 0)
        nlist_s = nr;
    __syncthreads();
    const int n_even = EO ? n_even_s : 0, n_odd = EO ? n_odd_s : 0;
    if (EO)
        c.vb = l_even;
    c.R = (EO ? n_even : c.nbg) * a.Ns;
    double* acoef = a.acoef + (long)c.g * nr * NK * NK * 2;
    auto AC = [&](int b, int i, int j) -> double* { return acoef + (((long)b * NK + i) * NK + j) * 2; };
    // y = A u (plain) or y = u - M_eo M_oe u on even blocks, the odd-block
    // intermediate in w2 (one more grid barrier), for the listed sources
    auto op = [&](const cpx<T>* u, cpx<T>* y, const int* lst, int nl) {
        if (EO) {
            apply_multi_mfma(c, a.Mt, 1, 9, l_odd, n_odd, u, (const cpx<T>*)nullptr, 0.0, 1.0, a.w2, lst, nl);
            grid_barrier(a.bar_count, a.bar_gen, bar_target, a.stats);
            apply_multi_mfma(c, a.Mt, 1, 9, l_even, n_even, (const cpx<T>*)a.w2, u, 1.0, -1.0, y, lst, nl);
        } else {
            apply_multi_mfma(c, a.At, 0, 9, (const int*)nullptr, c.nbg, u, (const cpx<T>*)nullptr, 0.0, 1.0, y, lst,
                             nl);
        }
    };
    // the system's right-hand sides: w, or w1_e - M_eo w1_o (w1 = M_0 w) on even blocks
    const cpx<T>* rhs = a.w;
    if (EO) {
        apply_multi_mfma(c, a.Mt, 0, 1, (const int*)nullptr, c.nbg, a.w, (const cpx<T>*)nullptr, 0.0, 1.0, a.w1,
                         list, nr);
        grid_barrier(a.bar_count, a.bar_gen, bar_target, a.stats);
        apply_multi_mfma(c, a.Mt, 1, 9, l_even, n_even, (const cpx<T>*)a.w1, (const cpx<T>*)a.w1, 1.0, -1.0, a.w2,
                         list, nr);
        rhs = a.w2;
    }

    // x = 0, r = rhs, ||rhs_b||^2
    for (long q = c.t; q < (long)c.R * nr; q += LT) {
        const int b = (int)(q / c.R), e = (int)(q - (long)b * c.R);
        const long i = c.entry(e) + b * N;
        a.x[i] = cpx<T>{0, 0};
        a.r[i] = rhs[i];
    }
    __syncthreads();
    multi_norm2(c, rhs, list, nr, SW);
    grid_barrier(a.bar_count, a.bar_gen, bar_target, a.stats);
    multi_reduce_real(a.part, nr, c.G, SW, list, nr, wn2);
    if (c.t < nr) {
        conv[c.t] = !(wn2[c.t] > 0.0);
        stop[c.t] = conv[c.t];
    }
    __syncthreads();
    int iters = 0;

    // every branch depends on values all workgroups reduce identically
    while (iters < a.maxiter) {
        if (c.t == 0) {
            int n = 0;
            for (int b = 0; b < nr; ++b) {
                act[b] = !stop[b];
                kb[b] = 0;
                if (act[b])
                    list[n++] = b;
            }
            nlist_s = n;
        }
        __syncthreads();
        if (nlist_s == 0)
            break;
        int k = 0;
        for (; k < a.nkv && iters < a.maxiter; ++k) {
            const int nl = nlist_s;
            // xi_k = r and the partial ||r||^2 for the RHS still in the cycle
            for (long q = c.t; q < (long)c.R * nl; q += LT) {
                const int bi = (int)(q / c.R), e = (int)(q - (long)bi * c.R);
                const int b = list[bi];
                const long i = c.entry(e);
                a.xi[((long)k * nr + b) * N + i] = a.r[b * N + i];
            }
            multi_norm2(c, a.r, list, nl, SC);
            grid_barrier(a.bar_count, a.bar_gen, bar_target, a.stats);  // S1
            multi_reduce_real(a.part, nr, c.G, SC, list, nl, rn2);
            if (c.t == 0) {
                int n = 0;
                for (int bi = 0; bi < nl; ++bi) {
                    const int b = list[bi];
                    if (k > 0 && rn2[b] <= tol2 * wn2[b])
                        act[b] = 0;  // converged with k directions
                    else
                        list[n++] = b;
                }
                nlist_s = n;
            }
            __syncthreads();
            const int na = nlist_s;
            if (na == 0)
                break;
            op(a.xi + (long)k * nr * N, a.chi + (long)k * nr * N, list, na);
            multi_pass(c, k, list, na, SA);
            grid_barrier(a.bar_count, a.bar_gen, bar_target, a.stats);  // S2
            multi_fin(a.part, a.fin, nr, c.G, c.g, SA, 2 * k + 2, list, na);
            grid_barrier(a.bar_count, a.bar_gen, bar_target, a.stats);  // S2b
            for (int q = c.t; q < na * (2 * k + 2) * 2; q += LT) {
                const int bi = q / ((2 * k + 2) * 2), rem = q - bi * (2 * k + 2) * 2;
                const int b = list[bi];
                red[b][rem] = a.fin[(long)b * RS * 2 + rem];
            }
            __syncthreads();
            if (c.t < na) {
                const int b = list[c.t];
                double n2 = red[b][4 * k];
                double b2 = n2;
                for (int j = 0; j < k; ++j)
                    b2 -= red[b][2 * j] * red[b][2 * j] + red[b][2 * j + 1] * red[b][2 * j + 1];
                second[b] = (k > 0 && !(b2 >= 0.01 * n2)) ? 1 : 0;
                for (int j = 0; j < k; ++j) {
                    double* p = AC(b, j, k);
                    p[0] = 0.0;
                    p[1] = 0.0;
                }
            }
            __syncthreads();
            if (c.t == 0) {
                int n = 0;
                for (int bi = 0; bi < na; ++bi)
                    if (second[list[bi]])
                        list2[n++] = list[bi];
                nlist2_s = n;
            }
            __syncthreads();
            const int n2l = nlist2_s;
            if (n2l > 0) {
                // heavy cancellation for some RHS: subtract the first projections, then a second pass
                for (long q = c.t; q < (long)c.R * n2l; q += LT) {
                    const int bi = (int)(q / c.R), e = (int)(q - (long)bi * c.R);
                    const int b = list2[bi];
                    const long i = c.entry(e);
                    cpx<T>* ck = a.chi + ((long)k * nr + b) * N;
                    double yr = (double)ck[i].re, yi = (double)ck[i].im;
                    for (int j = 0; j < k; ++j) {
                        cpx<T> z = a.chi[((long)j * nr + b) * N + i];
                        yr -= red[b][2 * j] * (double)z.re - red[b][2 * j + 1] * (double)z.im;
                        yi -= red[b][2 * j] * (double)z.im + red[b][2 * j + 1] * (double)z.re;
                    }
                    ck[i] = cpx<T>{(T)yr, (T)yi};
                }
                if (c.t < n2l) {
                    const int b = list2[c.t];
                    for (int j = 0; j < k; ++j) {
                        double* p = AC(b, j, k);
                        p[0] = red[b][2 * j];
                        p[1] = red[b][2 * j + 1];
                    }
                }
                __syncthreads();
                multi_pass(c, k, list2, n2l, SB);
                grid_barrier(a.bar_count, a.bar_gen, bar_target, a.stats);  // S3
                multi_fin(a.part, a.fin, nr, c.G, c.g, SB, 2 * k + 2, list2, n2l);
                grid_barrier(a.bar_count, a.bar_gen, bar_target, a.stats);  // S3b
                for (int q = c.t; q < n2l * (2 * k + 2) * 2; q += LT) {
                    const int bi = q / ((2 * k + 2) * 2), rem = q - bi * (2 * k + 2) * 2;
                    const int b = list2[bi];
                    red[b][rem] = a.fin[(long)b * RS * 2 + rem];
                }
                __syncthreads();
            }
            if (c.t < na) {
                const int b = list[c.t];
                double b2 = red[b][4 * k];
                double crr = red[b][4 * k + 2], cri = red[b][4 * k + 3];
                for (int j = 0; j < k; ++j) {
                    double ar = red[b][2 * j], ai = red[b][2 * j + 1];
                    double qr = red[b][2 * (k + j)], qi = red[b][2 * (k + j) + 1];
                    b2 -= ar * ar + ai * ai;
                    crr -= ar * qr + ai * qi;
                    cri -= ar * qi - ai * qr;
                    double* p = AC(b, j, k);
                    p[0] += ar;
                    p[1] += ai;
                }
                double bb = b2 > 0.0 ? sqrt(b2) : 0.0;
                bcoef[b][k] = bb;
                ccoef[b][k][0] = bb > 0.0 ? crr / bb : 0.0;
                ccoef[b][k][1] = bb > 0.0 ? cri / bb : 0.0;
            }
            __syncthreads();
            if (c.t == 0) {
                int n = 0;
                for (int bi = 0; bi < na; ++bi) {
                    const int b = list[bi];
                    if (!(bcoef[b][k] > 0.0)) {
                        act[b] = 0;  // new direction in the span: the RHS ends its cycle without it
                        stop[b] = 1;
                    } else {
                        kb[b] = k + 1;
                        list[n++] = b;
                    }
                }
                nlist_s = n;
            }
            __syncthreads();
            const int nu = nlist_s;
            for (long q = c.t; q < (long)c.R * nu; q += LT) {
                const int bi = (int)(q / c.R), e = (int)(q - (long)bi * c.R);
                const int b = list[bi];
                const long i = c.entry(e);
                cpx<T>* ck = a.chi + ((long)k * nr + b) * N;
                const double inv = 1.0 / bcoef[b][k], cr0 = ccoef[b][k][0], ci0 = ccoef[b][k][1];
                double yr = (double)ck[i].re, yi = (double)ck[i].im;
                for (int j = 0; j < k; ++j) {
                    cpx<T> z = a.chi[((long)j * nr + b) * N + i];
                    yr -= red[b][2 * j] * (double)z.re - red[b][2 * j + 1] * (double)z.im;
                    yi -= red[b][2 * j] * (double)z.im + red[b][2 * j + 1] * (double)z.re;
                }
                yr *= inv;
                yi *= inv;
                ck[i] = cpx<T>{(T)yr, (T)yi};
                cpx<T>* rb = a.r + b * N;
                double rr = (double)rb[i].re - (cr0 * yr - ci0 * yi);
                double ri = (double)rb[i].im - (cr0 * yi + ci0 * yr);
                rb[i] = cpx<T>{(T)rr, (T)ri};
            }
            ++iters;
            __syncthreads();
            if (nu == 0)
                break;
        }
        // x_b += sum alpha_j xi_j for the RHS that took directions in this cycle
        if (c.t < nr) {
            const int b = c.t;
            for (int i = kb[b] - 1; i >= 0; --i) {
                double sr = ccoef[b][i][0], si = ccoef[b][i][1];
                for (int j = i + 1; j < kb[b]; ++j) {
                    const double* p = AC(b, i, j);
                    sr -= p[0] * alpha[b][j][0] - p[1] * alpha[b][j][1];
                    si -= p[0] * alpha[b][j][1] + p[1] * alpha[b][j][0];
                }
                alpha[b][i][0] = sr / bcoef[b][i];
                alpha[b][i][1] = si / bcoef[b][i];
            }
        }
        if (c.t == 0) {
            int n = 0;
            for (int b = 0; b < nr; ++b)
                if (kb[b] > 0)
                    list[n++] = b;
            nlist_s = n;
        }
        __syncthreads();
        const int nx = nlist_s;
        for (long q = c.t; q < (long)c.R * nx; q += LT) {
            const int bi = (int)(q / c.R), e = (int)(q - (long)bi * c.R);
            const int b = list[bi];
            const long i = c.entry(e);
            double yr = (double)a.x[b * N + i].re, yi = (double)a.x[b * N + i].im;
            for (int j = 0; j < kb[b]; ++j) {
                cpx<T> z = a.xi[((long)j * nr + b) * N + i];
                yr += alpha[b][j][0] * (double)z.re - alpha[b][j][1] * (double)z.im;
                yi += alpha[b][j][0] * (double)z.im + alpha[b][j][1] * (double)z.re;
            }
            a.x[b * N + i] = cpx<T>{(T)yr, (T)yi};
        }
        // recompute r_b = w_b - A x_b for those RHS
        grid_barrier(a.bar_count, a.bar_gen, bar_target, a.stats);
        op(a.x, a.r, list, nx);
        for (long q = c.t; q < (long)c.R * nx; q += LT) {
            const int bi = (int)(q / c.R), e = (int)(q - (long)bi * c.R);
            const int b = list[bi];
            const long i = c.entry(e) + b * N;
            a.r[i] = cpx<T>{(T)((double)rhs[i].re - (double)a.r[i].re), (T)((double)rhs[i].im - (double)a.r[i].im)};
        }
        __syncthreads();
        multi_norm2(c, a.r, list, nx, SR);
        grid_barrier(a.bar_count, a.bar_gen, bar_target, a.stats);
        multi_reduce_real(a.part, nr, c.G, SR, list, nx, rn2);
        if (c.t < nx) {
            const int b = list[c.t];
            conv[b] = rn2[b] <= tol2 * wn2[b];
            if (conv[b])
                stop[b] = 1;
        }
        __syncthreads();
        if (nx == 0)
            break;  // no RHS made progress: all stopped
    }
    if (EO) {
        // x_o = w1_o - M_oe x_e for every source: a grid barrier followed the
        // last update of x_e (the zero start or the update before the residue
        // recomputation), so the neighbours' entries are complete
        __syncthreads();
        if (c.t < nr)
            list[c.t] = c.t;
        __syncthreads();
        apply_multi_mfma(c, a.Mt, 1, 9, l_odd, n_odd, (const cpx<T>*)a.x, (const cpx<T>*)a.w1, 1.0, -1.0, a.x, list,
                         nr);
    }
    if (c.g == 0 && c.t == 0) {
        int nc = 0;
        for (int b = 0; b < nr; ++b)
            nc += conv[b] ? 0 : 1;
        atomicAdd(&a.stats[0], iters);
        atomicAdd(&a.stats[1], nr);
        if (nc)
            atomicOr(&a.stats[2], 1);
    }
}

template <typename T>
void launch_impl(const Geom& g, int Ns, int nkv, int maxiter, double tol, const double* tol_dev, const cpx<T>* At,
                 const cpx<T>* Mt, const cpx<T>* Q, const cpx<T>* Z, int nq, int oblique, const double* Ainv,
                 const double* Gw, const cpx<T>* w, cpx<T>* x, cpx<T>* r,
                 cpx<T>* xi, cpx<T>* chi, cpx<T>* w1, cpx<T>* w2, double* part, int* stats, unsigned* bar_count,
                 unsigned long long* bar_gen, int grid_size, hipStream_t s, bool cooperative)
{
    LittleArgs<T> a;
    a.g = g;
    a.Ns = Ns;
    a.nkv = nkv;
    a.maxiter = maxiter;
    a.tol2 = tol * tol;
    a.tol_dev = tol_dev;
    a.At = At;
    a.Mt = Mt;
    a.w = w;
    a.x = x;
    a.r = r;
    a.xi = xi;
    a.chi = chi;
    a.w1 = w1;
    a.w2 = w2;
    a.Q = Mt ? Q : nullptr;
    a.Z = Mt ? Z : nullptr;
    a.nq = (Mt && Q && Z) ? nq : 0;
    a.oblique = oblique && a.nq > 0 && Ainv && Gw;
    a.Ainv = Ainv;
    a.Gw = Gw;
    if (oblique && a.nq > 0 && !a.oblique)
        fail(DFL_EINVAL, "oblique little deflation needs the inverse and Gram matrices");
    a.part = part;
    a.stats = stats;
    a.bar_count = bar_count;
    a.bar_gen = bar_gen;
    const void* fn = Mt ? reinterpret_cast<const void*>(&k_little_gcr<T, true>)
                        : reinterpret_cast<const void*>(&k_little_gcr<T, false>);
    if (!cooperative) {
        if (Mt)
            hipLaunchKernelGGL((k_little_gcr<T, true>), dim3(grid_size), dim3(LT1), 0, s, a);
        else
            hipLaunchKernelGGL((k_little_gcr<T, false>), dim3(grid_size), dim3(LT1), 0, s, a);
        HIPCHECK(hipGetLastError());
        return;
    }
    void* args[] = {&a};
    HIPCHECK(hipLaunchCooperativeKernel(fn, dim3(grid_size), dim3(LT1), args, 0, s));
}

}  // namespace

// The barrier and reduction costs grow with the workgroup count (a barrier
// takes about 2.2 us at 64 and 3.4 us at 128 workgroups on MI355X), the
// apply's bandwidth with it. Default four blocks per workgroup: with the
// even-odd operator each apply covers two blocks, one round of the 512
// threads for Ns up to 32 (measured on 16^4: 64 workgroups beat 32, 48 and
// 128). At most kLittleMaxGrid workgroups.
int little_gcr_grid(const Geom& g, int requested)
{
    int G = requested > 0 ? requested : g.Nb / 4;
    if (G > kLittleMaxGrid)
        G = kLittleMaxGrid;
    if (G > g.Nb)
        G = g.Nb;
    if (G < 1)
        G = 1;
    return G;
}

int little_gcr_multi_grid(const Geom& g, int requested)
{
    int G = requested > 0 ? 2 * requested : g.Nb / 4;
    if (G > kLittleMaxGridMulti)
        G = kLittleMaxGridMulti;
    if (G > g.Nb)
        G = g.Nb;
    if (G < 1)
        G = 1;
    return G;
}

int little_gcr_resident_limit(bool multi)
{
    int dev = 0, cus = 0;
    HIPCHECK(hipGetDevice(&dev));
    HIPCHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int per_cu = 1 << 30;
    auto occ = [&](const void* fn, int threads) {
        int n = 0;
        HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, threads, 0));
        per_cu = n < per_cu ? n : per_cu;
    };
    if (multi) {
        occ(reinterpret_cast<const void*>(&k_little_gcr_multi<double, false>), LT);
        occ(reinterpret_cast<const void*>(&k_little_gcr_multi<float, false>), LT);
        occ(reinterpret_cast<const void*>(&k_little_gcr_multi<double, true>), LT);
        occ(reinterpret_cast<const void*>(&k_little_gcr_multi<float, true>), LT);
    } else {
        occ(reinterpret_cast<const void*>(&k_little_gcr<double, true>), LT1);
        occ(reinterpret_cast<const void*>(&k_little_gcr<double, false>), LT1);
        occ(reinterpret_cast<const void*>(&k_little_gcr<float, true>), LT1);
        occ(reinterpret_cast<const void*>(&k_little_gcr<float, false>), LT1);
    }
    return per_cu * cus;
}

bool little_eo_fits(const Geom& g, int grid)
{
    return (g.Nb + grid - 1) / grid <= kMaxOwned;
}

size_t little_gcr_partial_doubles(int grid_size) { return (size_t)NSLOT * (grid_size + 1) * 2; }

template <typename T>
void launch_little_gcr(const Geom& g, int Ns, int nkv, int maxiter, double tol, const double* tol_dev, const cpx<T>* At,
                       const cpx<T>* Mt, cpx<T>* w1, cpx<T>* w2, const cpx<T>* Q, const cpx<T>* Z, int nq, int oblique,
                       const double* Ainv, const double* Gw, const cpx<T>* w,
                       cpx<T>* x, cpx<T>* r, cpx<T>* xi, cpx<T>* chi, double* part, int* stats, unsigned* bar_count,
                       unsigned long long* bar_gen, int grid, hipStream_t s, bool cooperative)
{
    launch_impl<T>(g, Ns, nkv, maxiter, tol, tol_dev, At, Mt, Q, Z, nq, oblique, Ainv, Gw, w, x, r, xi, chi, w1, w2, part,
                   stats, bar_count, bar_gen, grid, s, cooperative);
}

template <typename T>
void launch_little_gcr_multi(const Geom& g, int Ns, int nkv, int maxiter, double tol, const double* tol_dev, int nrhs,
                             const cpx<T>* At, const cpx<T>* Mt, cpx<T>* w1, cpx<T>* w2,
                             const cpx<T>* w, cpx<T>* x, cpx<T>* r, cpx<T>* xi, cpx<T>* chi, double* part, double* fin,
                             double* acoef, int* stats, unsigned* bar_count, unsigned long long* bar_gen, int grid,
                             hipStream_t s, bool cooperative)
{
    if (Mt && !(w1 && w2 && little_eo_fits(g, grid)))
        fail(DFL_EINVAL, "even-odd little solve: missing work vectors or too many blocks per workgroup");
    LittleMultiArgs<T> a;
    a.g = g;
    a.Ns = Ns;
    a.nkv = nkv;
    a.maxiter = maxiter;
    a.nrhs = nrhs;
    a.tol2 = tol * tol;
    a.tol_dev = tol_dev;
    a.At = At;
    a.Mt = Mt;
    a.w1 = w1;
    a.w2 = w2;
    a.w = w;
    a.x = x;
    a.r = r;
    a.xi = xi;
    a.chi = chi;
    a.part = part;
    a.fin = fin;
    a.acoef = acoef;
    a.stats = stats;
    a.bar_count = bar_count;
    a.bar_gen = bar_gen;
    if (!cooperative) {
        if (Mt)
            hipLaunchKernelGGL((k_little_gcr_multi<T, true>), dim3(grid), dim3(LT), 0, s, a);
        else
            hipLaunchKernelGGL((k_little_gcr_multi<T, false>), dim3(grid), dim3(LT), 0, s, a);
        HIPCHECK(hipGetLastError());
        return;
    }
    void* args[] = {&a};
    const void* fn = Mt ? reinterpret_cast<const void*>(&k_little_gcr_multi<T, true>)
                        : reinterpret_cast<const void*>(&k_little_gcr_multi<T, false>);
    HIPCHECK(hipLaunchCooperativeKernel(fn, dim3(grid), dim3(LT), args, 0, s));
}

size_t little_gcr_multi_doubles(int grid_size, int nrhs, size_t* fin, size_t* acoef)
{
    *fin = (size_t)nrhs * RS * 2;
    *acoef = (size_t)grid_size * nrhs * NK * NK * 2;
    return (size_t)NSLOT * nrhs * grid_size * 2;
}

#define INST_MULTI(T)                                                                                               \
    template void launch_little_gcr_multi<T>(const Geom&, int, int, int, double, const double*, int, const cpx<T>*,  \
                                             const cpx<T>*, cpx<T>*, cpx<T>*, const cpx<T>*,                        \
                                             cpx<T>*, cpx<T>*, cpx<T>*, cpx<T>*, double*, double*, double*, int*,    \
                                             unsigned*, unsigned long long*, int, hipStream_t, bool);
INST_MULTI(double)
INST_MULTI(float)
#undef INST_MULTI

template void launch_little_gcr<double>(const Geom&, int, int, int, double, const double*, const c64*, const c64*,
                                        c64*, c64*, const c64*, const c64*, int, int, const double*, const double*,
                                        const c64*, c64*, c64*, c64*, c64*, double*, int*, unsigned*,
                                        unsigned long long*, int, hipStream_t, bool);
template void launch_little_gcr<float>(const Geom&, int, int, int, double, const double*, const c32*, const c32*,
                                       c32*, c32*, const c32*, const c32*, int, int, const double*, const double*,
                                       const c32*, c32*, c32*, c32*, c32*, double*, int*, unsigned*,
                                       unsigned long long*, int, hipStream_t, bool);

}  // namespace dfl
