// Host-side internals of the solver library: the context, and the launchers
// each kernel file exports to the solver driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "dfl.h"

namespace dfl {

using c64 = cpx<double>;
using c32 = cpx<float>;

// error handling: thrown inside the library, caught at the C boundary
struct Error {
    int code;
    std::string msg;
};
[[noreturn]] void fail(int code, const std::string& msg);
void hip_check(hipError_t e, const char* what);
#define HIPCHECK(x) ::dfl::hip_check((x), #x)

// Raise a kernel's dynamic LDS limit to `bytes`, once per process (thread-safe;
// a failure leaves the flag unset and is reported by HIPCHECK).
inline void set_max_lds_once(std::once_flag& flag, const void* fn, int bytes)
{
    std::call_once(flag, [&] { HIPCHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)); });
}

// Schwarz block grid (independent of the layout blocks)
struct SapGeom {
    int sb[4];    // SAP block extent
    int nsb[4];   // SAP blocks per direction
    int lstr[4];  // in-block strides (lexicographic, y3 fastest)
    int Vsb;      // sites per SAP block
    int n_per_colour;
    int one_rl;   // one field: 1 = one lane per site, two blocks per CU (many blocks per colour),
                  // 0 = lane pairs, one block per CU
};

// links, two rows per matrix (the third is conj(row0 x row1)): FP64, FP32 and
// BF16 [4][6] entries per site in 64-site tiles
struct Links64 {
    const c64* u;
    long V;
};
struct Links32 {
    const c32* u;
    long V;
};
struct LinksBF16 {
    const uint32_t* u;
    long V;
};

// device scratch for reductions
constexpr int kRedBlocks = 480;   // fixed grid of the partial-sum kernels (deterministic)
constexpr int kRedThreads = 256;
constexpr int kMaxDot = 64;       // most vectors in one multi-dot
constexpr int kMaxLittleNkv = 32; // most Krylov vectors of the little GCR
constexpr int kLittleMaxGrid = 256;  // workgroups of the cooperative little GCR (one per CU)
constexpr int kMaxLittleRhs = 16;    // right-hand sides of one batched little solve
constexpr int kMaxLittleDefl = 32;   // global deflation directions of the little system
constexpr int kCloverComp = 36;         // complex entries of the clover term per site (two packed 6 x 6 blocks)
constexpr int kLittleMaxGridMulti = 256;  // workgroups of the batched little GCR (one per CU)

}  // namespace dfl

struct dfl_ctx {
    dfl_params p;
    hipStream_t stream = nullptr;
    int device = 0;
    dfl::Geom g;
    dfl::SapGeom sg;
    long V = 0;
    long field_elems = 0;  // complex entries of one quark field (12 V)

    // gauge field
    dfl::c64* U64 = nullptr;
    dfl::c32* U32 = nullptr;
    uint32_t* Ubf = nullptr;
    dfl::c64* Cl64 = nullptr;  // clover term (csw != 0), FP64 and FP32, 36 complex per site
    dfl::c32* Cl32 = nullptr;
    bool have_gauge = false;

    // deflation subspace
    dfl::c64* Phi = nullptr;   // [Ns][12][V]
    dfl::c32* Phi32 = nullptr; // FP32 copy (inner projections in mixed precision)
    dfl::c64* A64 = nullptr;   // [Nb][9][Ns][Ns] at m0_A
    dfl::c32* A32 = nullptr;   // FP32 copy, same layout
    dfl::c64* At64 = nullptr;  // blocks transposed, [Nb][9][l][k] (little GCR kernel)
    dfl::c32* At32 = nullptr;
    dfl::c64* Mt64 = nullptr;  // even-odd little system: D^-1 and D^-1 A_d, transposed blocks
    dfl::c32* Mt32 = nullptr;
    bool eo_ok = false;        // Mt is current and every diagonal block was safely invertible
    dfl::c64* gsR = nullptr;   // block Gram-Schmidt coefficients [Nb][Ns][Ns]
    dfl::c64* gU = nullptr;    // global deflation of the little system: Ns vectors each
    dfl::c64* gW = nullptr;
    dfl::c64* gQ = nullptr;
    dfl::c64* gZ = nullptr;
    dfl::c32* gQ32 = nullptr;
    dfl::c32* gZ32 = nullptr;
    dfl::c64* gC = nullptr;    // Ns x Ns scratch (Gram matrix, transform)
    double* gAinv = nullptr;   // oblique form: (Z^+ A_hat Z)^-1 and W^+ W, Ns x Ns complex each
    double* gGw = nullptr;
    int gdefl_n = 0;           // deflation directions in use (0: none)
    bool gdefl_oblique = false;
    double m0_A = 0.0;
    bool have_subspace = false;

    // FP64 field workspaces
    dfl::c64* xi = nullptr;    // nkv Krylov directions
    dfl::c64* chi = nullptr;   // nkv orthonormal images
    dfl::c64* rho = nullptr;
    dfl::c64* acc = nullptr;
    dfl::c64* t1 = nullptr;
    dfl::c64* t2 = nullptr;
    dfl::c64* t3 = nullptr;
    // FP32 SAP workspaces
    dfl::c32* s32a = nullptr;
    dfl::c32* s32b = nullptr;
    dfl::c32* s32c = nullptr;
    dfl::c64* tN = nullptr;    // Ns FP64 fields: FP64 inverse-iteration output
    dfl::c64* bootF = nullptr; // bootstrapped inverse iteration: the Ns fields and
    dfl::c64* bootT = nullptr; //   their coarse parts Phi A^-1 Phi^+ psi
    // little-system workspaces (max(FP64) size; reused for FP32)
    void* lxi = nullptr;
    void* lchi = nullptr;
    void* lr = nullptr;
    void* lx = nullptr;
    void* lw = nullptr;
    void* lt = nullptr;
    void* lw1 = nullptr;       // even-odd workspaces of the little GCR
    void* lw2 = nullptr;
    dfl::c32* lw32 = nullptr;  // FP32 little source and solution (mixed precision)
    dfl::c32* lx32 = nullptr;
    double* lpart = nullptr;   // partial sums of the cooperative little GCR
    int* lstats = nullptr;     // [iterations, solves, failure flags, spare]
    unsigned* lbar_count = nullptr;         // grid barrier of the little GCR kernel
    unsigned long long* lbar_gen = nullptr;
    int lgrid = 0;             // its grid size
    int lgrid_multi = 0;       // grid of the batched little GCR
    double* lfin = nullptr;    // batched little GCR: reduced sums and per-workgroup coefficients
    double* lacoef = nullptr;
    // reductions and scalars
    double* red = nullptr;       // kRedBlocks * 2 * kMaxDot partials per field (max(nrhs_max, multi-field count))
    double* dnorm = nullptr;     // squared norms (complex pairs) of the fields of a multi-field normalisation
    double* dscal = nullptr;     // device scalars
    double* hscal = nullptr;     // pinned host mirror
    int* dflag = nullptr;        // device status flag
    int* dact = nullptr;         // per-RHS active mask of the batched GCR
    int* dact2 = nullptr;        // per-RHS mask of the outer GCR's second Gram-Schmidt pass
    double* dtol = nullptr;      // relative tolerance of the inner little solves (device)
    double* htol = nullptr;      // pinned host mirror
    int* hact = nullptr;         // pinned host mirror
    size_t alloc_bytes = 0;
    std::vector<double> history;  // outer GCR residues of the last solve
    // start-field network scratch (grown on demand)
    float* net_part = nullptr;   // weight-gradient partial sums
    size_t net_part_n = 0;
    uint16_t* net_wbf = nullptr; // BF16 weights of the BF16 forward
    size_t net_wbf_n = 0;
    dfl::c64* PhiT = nullptr;    // the basis in the transposed in-block order (assembly of the
    size_t PhiT_n = 0;           // face columns along x2 and x3)
    dfl::c64* loss_Y = nullptr;  // deficit loss: per-block G^-1 Psi^+ T
    double* loss_buf = nullptr;  // [Nb][K] block norms, [Nb][K] projections, [K] weights
    double* loss_host = nullptr;
    size_t loss_n = 0;
    // HIP graphs of the GCR steps, keyed by (step index, number of sources)
    bool use_graph = false;
    bool capturing = false;
    hipStream_t gstream = nullptr;     // capture and replay stream, fenced to `stream` by events
    hipEvent_t gev[2] = {nullptr, nullptr};
    std::vector<std::pair<long, hipGraphExec_t>> graphs;
    long graph_replays = 0;
    // kernel-class timers
    double t_setup_last = 0.0;  // seconds of the last dfl_setup
    bool prof_on = false;
    int sap_prof_cls = DFL_PROF_SAP;  // class the Schwarz sweeps are timed in (setup during inverse iteration)
    std::vector<hipEvent_t> ev_pool;                 // free events
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
    double prof_t[8] = {0};
    long long prof_n[8] = {0};
    long long prof_little_iters = 0;
};

namespace dfl {

// ---------------------------------------------------------------- layout.hip
void launch_pack_field64(const Geom& g, const c64* canon, c64* nat, int nrhs, hipStream_t s);
void launch_pack_field32(const Geom& g, const c64* canon, c32* nat, int nrhs, hipStream_t s);
void launch_unpack_field64(const Geom& g, const c64* nat, c64* canon, int nrhs, hipStream_t s);
void launch_unpack_field32(const Geom& g, const c32* nat, c64* canon, int nrhs, hipStream_t s);
// flag |= 1 if some link's third row is not conj(row0 x row1)
void launch_pack_gauge(const Geom& g, const c64* canon, c64* U64, c32* U32, uint32_t* Ubf, int* flag, hipStream_t s);
void launch_f64_to_f32(const c64* in, c32* out, long n, hipStream_t s);
// nb fields of n entries: out_b = in_b / sqrt(nrm2[b * cstride]) in FP32
// (finite_flag non-null: bit 1 set there if an input entry is not finite)
void launch_f64_to_f32_scaled(const c64* in, c32* out, long n, int nb, const double* nrm2, int cstride, hipStream_t s,
                              int* finite_flag = nullptr);
void launch_f32_to_f64(const c32* in, c64* out, long n, hipStream_t s);

// ----------------------------------------------------------------- dirac.hip
// out = D psi (nrhs fields, each 12 V). mode 0: full D; 1: block-diagonal part
// (hops leaving a layout block dropped); 2: block-crossing hop in direction
// mu, orientation dir (no mass term).
// clov (may be null): the clover term (36 complex per site, see hop.h), in modes 0 and 1
void launch_dirac64(const Geom& g, Links64 U, const c64* psi, c64* out, int nrhs, double m0,
                    int mode, int mu, int dir, hipStream_t s, const c64* clov);
// out = sub - D psi (full operator, FP64) for nrhs fields; out aliases neither sub nor psi
void launch_dirac64_sub(const Geom& g, Links64 U, const c64* sub, const c64* psi, c64* out, int nrhs, double m0,
                        hipStream_t s, const c64* clov);
// MODE 2 on the face sites only (other sites of out untouched)
// transposed: psi and out in the transposed in-block order (site_compose_t)
void launch_dirac64_face(const Geom& g, Links64 U, const c64* psi, c64* out, int nrhs, int mu, int dir, hipStream_t s,
                         bool transposed = false);
// dst = src with every block's sites in the transposed in-block order (nf FP64 fields)
void launch_to_transposed(const Geom& g, const c64* src, c64* dst, int nf, hipStream_t s);
void launch_dirac32(const Geom& g, Links32 U, const c32* psi, c32* out, int nrhs, float m0, hipStream_t s,
                    const c32* clov);
void launch_dirac_bf16(const Geom& g, LinksBF16 U, const c32* psi, c32* out, int nrhs, float m0, hipStream_t s,
                       const c32* clov);
// clover term of the O(a)-improved operator from the FP64 links: csw (i/4)
// sum_{mu,nu} sigma_{mu nu} Fhat_{mu nu}(x), stored per chirality block (hop.h)
// in FP64 (C64) and FP32 (C32, may be null)
void launch_clover_field(const Geom& g, Links64 U, double csw, c64* C64, c32* C32, hipStream_t s);

// ------------------------------------------------------------------- sap.hip
// one colour sweep for nrhs fields (each 12 V entries, back to back)
// init: 0 = general psi, 1 = psi zero on the sweep's own blocks, 2 = psi
// zero everywhere (the two sweeps of the first cycle); out64 (FP32 sweeps,
// may be null): the blocks' new psi also written there in FP64
// clov (may be null): the clover term in the sweep's precision
void launch_sap_colour64(const Geom& g, const SapGeom& sg, Links64 U, const c64* rho, c64* psi,
                         double m0, int nmr, int colour, int nrhs, int init, hipStream_t s, const c64* clov);
// rho_nrm2 (may be null): field b of rho enters divided by sqrt(rho_nrm2[2 b])
void launch_sap_colour32(const Geom& g, const SapGeom& sg, Links32 U, const c32* rho, c32* psi,
                         float m0, int nmr, int colour, int nrhs, int init, c64* out64, hipStream_t s,
                         const c32* clov, const double* rho_nrm2 = nullptr);
void launch_sap_colour_bf16(const Geom& g, const SapGeom& sg, LinksBF16 U, const c32* rho, c32* psi,
                            float m0, int nmr, int colour, int nrhs, int init, c64* out64, hipStream_t s,
                            const c32* clov, const double* rho_nrm2 = nullptr);

// ------------------------------------------------------------------ blas.hip
template <typename T> void launch_zero(cpx<T>* x, long n, hipStream_t s);
template <typename T> void launch_copy(const cpx<T>* x, cpx<T>* y, long n, hipStream_t s);
// z = x + y
template <typename T> void launch_add(const cpx<T>* x, const cpx<T>* y, cpx<T>* z, long n, hipStream_t s);
// z = x - y
template <typename T> void launch_sub(const cpx<T>* x, const cpx<T>* y, cpx<T>* z, long n, hipStream_t s);
// out[j] = (X_j, y) for j < m, X_j = X + j*stride; complex results to dst (2 doubles each)
template <typename T>
void launch_multidot(const cpx<T>* X, long stride, int m, const cpx<T>* y, long n, double* red,
                     double* dst, hipStream_t s);
// dst = ||x||^2
template <typename T> void launch_norm2(const cpx<T>* x, long n, double* red, double* dst, hipStream_t s);
// y += sign * sum_j coef[j] X_j  (coef: m complex doubles on the device)
template <typename T>
void launch_multiaxpy(const cpx<T>* X, long stride, int m, const double* coef, double sign, cpx<T>* y,
                      long n, hipStream_t s);
// x *= 1/sqrt(*nrm2)
template <typename T> void launch_scale_invsqrt(cpx<T>* x, long n, const double* nrm2, hipStream_t s);
// Batched forms over nb right-hand sides: RHS b's vectors at offsets b*xb
// (X, x) and b*yb (y), its scalars at b*cstride / b*dstride; RHS with
// active[b] == 0 are skipped when active is non-null. red holds kMaxDot *
// kRedBlocks * 2 doubles per RHS.
template <typename T>
void launch_multidot_b(const cpx<T>* X, long stride, int m, const cpx<T>* y, long n, int nb, long xb, long yb,
                       double* red, double* dst, int dstride, const int* active, hipStream_t s);
template <typename T>
void launch_norm2_b(const cpx<T>* x, long n, int nb, long xb, double* red, double* dst, int dstride,
                    const int* active, hipStream_t s);
template <typename T>
void launch_multiaxpy_b(const cpx<T>* X, long stride, int m, const double* coef, int cstride, double sign, cpx<T>* y,
                        long n, int nb, long xb, long yb, const int* active, hipStream_t s);
// GCR closing steps (FP64): dst[b*dstride + 0..3] = {||x_b||^2, 0, (x_b, y_b)};
// then y_b -= ((x_b, y_b) / ||x_b||^2) x_b, x_b /= ||x_b|| with those sums (sc),
// and dst[b*dstride + 0..1] = {||y_b||^2, 0}. red: partial-sum scratch.
void launch_norm_dot_b(const c64* x, const c64* y, long n, int nb, long xb, double* red, double* dst, int dstride,
                       const int* active, hipStream_t s);
void launch_scale_update_b(c64* x, c64* y, long n, int nb, long xb, const double* sc, int cstride, double* red,
                           double* dst, int dstride, const int* active, hipStream_t s);
template <typename T>
void launch_scale_invsqrt_b(cpx<T>* x, long n, int nb, long xb, const double* nrm2, int cstride, const int* active,
                            hipStream_t s);
// second Gram-Schmidt pass only where the first cancelled > 99% of ||y||^2:
// act2[b] set accordingly, a2 zeroed for the sources that skip it (nb <= 64)
void launch_second_pass_mask(const double* a1, double* a2, int k, int stride, const int* active, int nb, int* act2,
                             hipStream_t s);
// dst[0..1] = a[0..1] + b[0..1] for m complex
void launch_add_scalars(const double* a, const double* b, double* dst, int m, hipStream_t s);
// finite check: flag |= 1 if any entry of x is NaN or Inf
template <typename T> void launch_finite_check(const cpx<T>* x, long n, int* flag, hipStream_t s);

// ------------------------------------------------------------------- dfl.hip
// w_b[blk][k] = (Phi_k, psi_b) over each layout block, nrhs fields (little
// vectors of Nb*Ns entries back to back)
void launch_restrict64(const Geom& g, const c64* Phi, int Ns, const c64* psi, c64* w, int nrhs, hipStream_t s);
// psi_b = sum_k Phi_k v_b[blk][k]
void launch_prolong64(const Geom& g, const c64* Phi, int Ns, const c64* v, c64* psi, int nrhs, hipStream_t s);
// the same with an FP32 copy of the basis (FP64 fields, FP64 arithmetic)
void launch_restrict_b32(const Geom& g, const c32* Phi, int Ns, const c64* psi, c64* w, int nrhs, hipStream_t s);
void launch_prolong_b32(const Geom& g, const c32* Phi, int Ns, const c64* v, c64* psi, int nrhs, hipStream_t s);
// block Gram-Schmidt in place on Ns fields (modified GS, order l = 0..Ns-1);
// R (may be null): [Nb][Ns][Ns] coefficients, field l = sum_k R[k][l] basis k
// FT, F32 (may be null): the result also in the transposed in-block order
// (site_compose_t) and in FP32; returns whether those copies were written (the
// 256-site block kernel writes them, the caller makes them otherwise)
bool launch_block_gs64(const Geom& g, c64* F, int Ns, double rank_tol, int* flag, c64* R, hipStream_t s,
                       c64* FT = nullptr, c32* F32 = nullptr);
// global modes of the little system from R: Ns little vectors, even blocks only
void launch_global_modes(const Geom& g, const c64* R, int Ns, c64* U, hipStream_t s);
// on blocks of the given parity: out = alpha sv + beta sum_{d>=1} (D^-1 A_d) in_{nbr} (nv vectors)
void launch_eo_hop(const Geom& g, const c64* Mt, int Ns, const c64* in, const c64* sv, c64* out, int nv, int parity,
                   double alpha, double beta, hipStream_t s);
// G[k][l] = (X_k, X_l); Y_l = sum_k X_k C[k][l] for l < m (C is nv x m)
void launch_gram(const c64* X, long n, int nv, c64* G, hipStream_t s);
// G[k][l] = (X_k, Y_l) for k, l < nv
void launch_gram2(const c64* X, const c64* Y, long n, int nv, c64* G, hipStream_t s);
void launch_combine(const c64* X, long n, int nv, int m, const c64* C, c64* Y, hipStream_t s);
// A[blk][d][k][l0 + j] = (Phi_k, Y_j) over each block for k < Ns, j < nc
// (nc <= little_columns_max(Ns), nc + Ns <= 128); part: scratch of part_cap
// complex entries for the split partial sums (at least Nb*Ns*nc). transposed
// (face columns d > 0 with little_columns_transposable only): Phi and Y in
// the transposed in-block order (site_compose_t).
int little_columns_max(int Ns);
bool little_columns_transposable(int Ns, int nc);
void launch_little_columns64(const Geom& g, const c64* Phi, int Ns, const c64* Y, int nc, int l0, int d, c64* A,
                             c64* part, long part_cap, hipStream_t s, bool transposed = false);
// All Ns columns of direction d in one launch on the matrix cores (Ns <= 32,
// part_cap >= Nb Ns^2): columns j < n1 of Y1, the others of Y2 (Ns - n1
// fields); transposed as for launch_little_columns64 (face columns only).
bool little_columns_all_ok(int Ns, long part_cap, long Nb);
void launch_little_columns64_all(const Geom& g, const c64* Phi, int Ns, const c64* Y1, int n1, const c64* Y2, int d,
                                 c64* A, c64* part, long part_cap, hipStream_t s, bool transposed);
// w_b = A v_b (9-point block stencil) for nrhs little vectors
template <typename T>
void launch_little_apply(const Geom& g, const cpx<T>* A, int Ns, const cpx<T>* v, cpx<T>* w, int nrhs, hipStream_t s);
// the same in FP32 on the matrix cores, from the transposed blocks At
void launch_little_apply_mfma(const Geom& g, const c32* At, int Ns, const c32* v, c32* w, int nrhs, hipStream_t s);
// A[blk][0][k][k] += dm  (mass shift)
void launch_little_shift(const Geom& g, c64* A, int Ns, double dm, hipStream_t s);
void launch_c64_to_c32(const c64* a, c32* b, long n, hipStream_t s);
// Even-odd preparation (appendix A.2): per block D^-1 of the diagonal block by
// Gauss-Jordan elimination with partial pivoting, and M_d = D^-1 A_d for the
// eight neighbour terms; stored transposed like At: Mt[blk][0] = D^-1,
// Mt[blk][d] = M_d. flag |= 1 when a pivot is below 1e-8 of the block's
// largest entry (the caller then keeps the plain system).
void launch_little_eo_prep(const Geom& g, const c64* A, int Ns, c64* Mt64, c32* Mt32, int* flag, hipStream_t s);
// A32 = A, At64 = At32 = A with every Ns x Ns block transposed
void launch_little_copies(const c64* A, c32* A32, c64* At64, c32* At32, long nblocks, int Ns, hipStream_t s);

// ------------------------------------------------------------------- net.hip
// Start-field network: FP32 planes [C][V] in canonical site order.
void launch_net_features(const Geom& g, const c64* U64, const float* noise, float* x, hipStream_t s);
void launch_conv_forward(const Geom& g, const float* in, int cin, const float* W, const float* b, int cout, float* z,
                         float* a, hipStream_t s);
size_t conv_wgrad_chunk_floats(const Geom& g, int cin, int cout, long* chunk, int* nchunk);
// BF16-operand forward (FP32 sums) for lattices with L3 % 32 == 0 and L2 % 4 == 0
// (conv_bf16_fits); Wb holds conv_bf16_weight_elems(cin, cout) BF16 entries
bool conv_bf16_fits(const Geom& g);
size_t conv_bf16_weight_elems(int cin, int cout);
void launch_conv_forward_bf16(const Geom& g, const float* in, int cin, const float* W, const float* b, int cout,
                              float* z, float* a, uint16_t* Wb, hipStream_t s);
void launch_conv_backward(const Geom& g, const float* in, int cin, const float* W, int cout, const float* gr,
                          float* dW, float* db, float* din, const float* zprev, float* part, long chunk, int nchunk,
                          hipStream_t s);
void launch_out_to_fields(const Geom& g, const float* out, int Ns, c64* f, hipStream_t s);
void launch_fields_to_out(const Geom& g, const c64* gr, int Ns, float* dout, hipStream_t s);
void launch_deficit_block(const Geom& g, const c64* Psi, int Ns, const c64* T, int K, c64* Y, double* tb2,
                          double* proj, int* flag, hipStream_t s);
void launch_deficit_grad(const Geom& g, const c64* Psi, int Ns, const c64* T, int K, const c64* Y, const double* wk,
                         c64* grad, hipStream_t s);
void launch_adam(float* th, const float* gr, float* m, float* v, long n, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t s);
// allocation-free weight gradient: floats of the device scratch array (64 MiB
// per device), its device address on the current device, and a chunking of
// the partial sums that fits cap floats (false if one chunk does not fit)
constexpr size_t kNoAllocFloats = size_t(16) << 20;
constexpr int kMaxDevices = 64;
float* noalloc_scratch();
bool conv_wgrad_chunk_fit(const Geom& g, int cin, int cout, size_t cap, long* chunk, int* nchunk);
constexpr int kNetMaxCin = 96;     // input channels of a convolution (weight gradient bound)
constexpr int kNetMaxCout = 576;   // output channels (input-gradient staging bound)
constexpr int kLossMaxN = 32;      // fields and targets of the deficit loss

// ---------------------------------------------------------------- little.hip
// workgroups of the little GCR: requested (0: Nb / 4), clamped to 1..min(Nb, kLittleMaxGrid)
int little_gcr_grid(const Geom& g, int requested);
size_t little_gcr_partial_doubles(int grid_size);
// workgroups of the batched little GCR: twice the requested single-source
// grid (0: Nb / 4), at most one per compute unit and the block count
int little_gcr_multi_grid(const Geom& g, int requested);
// workgroups of the (batched) little GCR kernels that can be resident at once
// on the current device (occupancy x compute units); the grid barrier needs
// the whole grid resident, also when the kernel is a graph node
int little_gcr_resident_limit(bool multi);
// whether the even-odd solver's per-workgroup block lists fit for this grid
bool little_eo_fits(const Geom& g, int grid);
// v = A^{-1} w by GCR to ||w - A v|| <= tol ||w|| in one cooperative launch
// (tol read from device memory at tol_dev when that is not null);
// r, xi, chi are workspaces; stats accumulates [iterations, solves, failed]
// With Mt non-null the GCR runs on the even-odd reduced system (appendix
// A.2) using the matrices of launch_little_eo_prep and the workspaces w1, w2
// (N entries each); otherwise on A itself. With nq > 0 (even-odd only) it is
// deflated by the nq orthonormal little vectors Q = A_hat Z (appendix A.3).
// cooperative = false launches it as an ordinary kernel (for graph capture):
// the grid (at most kLittleMaxGrid workgroups, one per compute unit) is then
// resident by construction when nothing else runs on the device, and the
// barriers' bounded polling reports a failure rather than hang otherwise.
// oblique = 1: section 3's projectors on the even-odd system instead (Q holds
// W = A_hat Z, Z orthonormal, Ainv = (Z^+ W)^-1 and Gw = W^+ W, nq x nq
// complex row-major on the device).
template <typename T>
void launch_little_gcr(const Geom& g, int Ns, int nkv, int maxiter, double tol, const double* tol_dev,
                       const cpx<T>* At, const cpx<T>* Mt, cpx<T>* w1, cpx<T>* w2, const cpx<T>* Q, const cpx<T>* Z,
                       int nq, int oblique, const double* Ainv, const double* Gw, const cpx<T>* w,
                       cpx<T>* x, cpx<T>* r, cpx<T>* xi, cpx<T>* chi, double* part, int* stats, unsigned* bar_count,
                       unsigned long long* bar_gen, int grid, hipStream_t s, bool cooperative = true);

// The same for nrhs systems at once (nrhs <= kMaxLittleRhs): w, x, r hold
// nrhs little vectors back to back, xi and chi nkv * nrhs. Sizes of part,
// fin and acoef (doubles) come from little_gcr_multi_doubles. With Mt
// non-null each system is solved in its even-odd reduced form (appendix A.2;
// w1 and w2 hold nrhs vectors each, little_eo_fits must hold for the grid);
// global-mode deflation is not applied here.
size_t little_gcr_multi_doubles(int grid_size, int nrhs, size_t* fin, size_t* acoef);
template <typename T>
void launch_little_gcr_multi(const Geom& g, int Ns, int nkv, int maxiter, double tol, const double* tol_dev, int nrhs,
                             const cpx<T>* At, const cpx<T>* Mt, cpx<T>* w1, cpx<T>* w2,
                             const cpx<T>* w, cpx<T>* x, cpx<T>* r, cpx<T>* xi, cpx<T>* chi, double* part, double* fin,
                             double* acoef, int* stats, unsigned* bar_count, unsigned long long* bar_gen, int grid,
                             hipStream_t s, bool cooperative = true);

}  // namespace dfl
