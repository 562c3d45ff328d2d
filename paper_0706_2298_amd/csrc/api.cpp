// C ABI of the solver library: context management, argument checks, and the
// host-side drivers of the Krylov solvers. All arithmetic runs in the HIP
// kernels of the other translation units; the host only sequences launches on
// the context's stream, reads back one block of scalars per Krylov step and
// solves the small triangular systems of GCR.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <exception>
#include <functional>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "dfl_net.h"

namespace dfl {

namespace {
thread_local std::string g_last_error;
}

void fail(int code, const std::string& msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char* what)
{
    if (e != hipSuccess)
        fail(e == hipErrorOutOfMemory ? DFL_ENOMEM : DFL_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

using cd = std::complex<double>;

// device scalar slots (doubles)
constexpr int S_A1 = 0;      // 64 complex: first Gram-Schmidt pass
constexpr int S_A2 = 128;    // 64 complex: second pass
constexpr int S_B = 256;     // ||chi_k||^2
constexpr int S_C = 258;     // (chi_k, rho) with chi_k before its normalisation
constexpr int S_R = 260;     // ||rho||^2
constexpr int S_DOWN = 264;  // doubles read back per step
constexpr int S_ALPHA = 512; // 64 complex: GCR solution coefficients
constexpr int S_TOTAL = 1024;

template <typename T> T* alloc_dev(dfl_ctx* c, size_t n)
{
    if (n == 0)
        return nullptr;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess)
        fail(DFL_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
    c->alloc_bytes += n * sizeof(T);
    return static_cast<T*>(p);
}

void free_all(dfl_ctx* c)
{
    void* ptrs[] = {c->U64, c->U32,  c->Ubf,  c->Phi, c->Phi32, c->A64, c->A32, c->xi,  c->chi,
                    c->rho, c->acc,  c->t1,   c->t2,  c->t3,    c->s32a, c->s32b, c->s32c, c->lxi,
                    c->lchi, c->lr,  c->lx,   c->lw,  c->lt,    c->lw32, c->lx32, c->red, c->dscal, c->dflag,
                    c->At64, c->At32, c->lpart, c->lstats, c->lbar_count, c->lbar_gen, c->tN,
                    c->lfin, c->lacoef, c->dact, c->net_part, c->loss_Y, c->loss_buf, c->dtol, c->Mt64, c->Mt32, c->lw1, c->lw2,
                    c->gsR, c->gU, c->gW, c->gQ, c->gZ, c->gQ32, c->gZ32, c->gC, c->Cl64, c->Cl32,
                    c->gAinv, c->gGw, c->bootF, c->bootT, c->net_wbf, c->PhiT};
    for (void* p : ptrs)
        if (p)
            (void)hipFree(p);
    if (c->hscal)
        (void)hipHostFree(c->hscal);
    if (c->hact)
        (void)hipHostFree(c->hact);
    if (c->loss_host)
        (void)hipHostFree(c->loss_host);
    if (c->htol)
        (void)hipHostFree(c->htol);
}

void check_blocks(const int dims[4], const int b[4], const char* what)
{
    for (int mu = 0; mu < 4; ++mu) {
        if (b[mu] < 1 || dims[mu] % b[mu] != 0)
            fail(DFL_EINVAL, std::string(what) + " block does not divide the lattice");
        int nb = dims[mu] / b[mu];
        if (nb < 2 || nb % 2 != 0)
            fail(DFL_EINVAL, std::string(what) + " block count per direction must be even and >= 2");
    }
}

void validate(const dfl_params& p)
{
    for (int mu = 0; mu < 4; ++mu)
        if (p.dims[mu] < 2)
            fail(DFL_EINVAL, "lattice extent must be >= 2 in every direction");
    double V = (double)p.dims[0] * p.dims[1] * p.dims[2] * p.dims[3];
    // 64-site tiles; 32-bit byte offsets into the FP64 link array (36 x 16 B per site)
    if (V > 4194304.0)
        fail(DFL_EINVAL, "lattice volume must be at most 2^22 sites");
    if (std::fmod(V, 64.0) != 0.0)
        fail(DFL_EINVAL, "lattice volume must be a multiple of 64 sites");
    check_blocks(p.dims, p.sap_block, "SAP");
    check_blocks(p.dims, p.dfl_block, "deflation");
    int vsb = p.sap_block[0] * p.sap_block[1] * p.sap_block[2] * p.sap_block[3];
    if (vsb > 512)
        fail(DFL_EINVAL, "SAP block volume must be <= 512 sites");
    int vb = p.dfl_block[0] * p.dfl_block[1] * p.dfl_block[2] * p.dfl_block[3];
    if (p.Ns < 1 || p.Ns > 64 || p.Ns > 12 * vb)
        fail(DFL_EINVAL, "Ns must be in 1..min(64, 12*|deflation block|)");
    if (p.ncy < 1 || p.nmr < 1)
        fail(DFL_EINVAL, "ncy and nmr must be >= 1");
    if (p.nkv < 1 || p.nkv > kMaxDot)
        fail(DFL_EINVAL, "nkv must be in 1..64");
    if (p.little_nkv < 1 || p.little_nkv > kMaxLittleNkv)
        fail(DFL_EINVAL, "little_nkv must be in 1..32");
    if (p.n_inviter < 0 || p.maxiter < 1 || p.little_maxiter < 1 || p.nrhs_max < 1)
        fail(DFL_EINVAL, "n_inviter >= 0, maxiter >= 1, little_maxiter >= 1, nrhs_max >= 1 required");
    if (p.little_grid < 0)
        fail(DFL_EINVAL, "little_grid must be >= 0");
    if (p.nrhs_max > kMaxLittleRhs)
        fail(DFL_EINVAL, "nrhs_max must be at most " + std::to_string(kMaxLittleRhs));
    if (!(p.tol > 0.0) || !(p.little_tol_in > 0.0) || !(p.little_tol_out > 0.0))
        fail(DFL_EINVAL, "tolerances must be positive");
    if (!std::isfinite(p.m0) || !std::isfinite(p.m0_setup))
        fail(DFL_EINVAL, "masses must be finite");
    if (p.link_prec < DFL_F64 || p.link_prec > DFL_BF16)
        fail(DFL_EINVAL, "link_prec must be F64, F32 or BF16");
    if (p.sap_prec != DFL_F64 && p.sap_prec != DFL_F32)
        fail(DFL_EINVAL, "sap_prec must be F64 or F32");
    if (p.sap_prec == DFL_F64 && p.link_prec != DFL_F64)
        fail(DFL_EINVAL, "FP64 SAP needs FP64 links");
    if (p.little_prec != DFL_F64 && p.little_prec != DFL_F32)
        fail(DFL_EINVAL, "little_prec must be F64 or F32");
    if (p.little_gdefl < 0 || p.little_gdefl > 2)
        fail(DFL_EINVAL, "little_gdefl must be 0, 1 or 2");
    if (p.n_boot < 0 || p.n_boot > p.n_inviter)
        fail(DFL_EINVAL, "n_boot must lie in 0..n_inviter");
    if (p.solver < DFL_SOLVER_GCR || p.solver > DFL_SOLVER_DFL_SAP_GCR)
        fail(DFL_EINVAL, "unknown solver");
    if (!std::isfinite(p.csw))
        fail(DFL_EINVAL, "csw must be finite");
    if (p.antiperiodic != 0 && p.antiperiodic != 1)
        fail(DFL_EINVAL, "antiperiodic must be 0 or 1");
}

Links64 links64(const dfl_ctx* c) { return Links64{c->U64, c->V}; }
Links32 links32(const dfl_ctx* c) { return Links32{c->U32, c->V}; }
LinksBF16 linksbf(const dfl_ctx* c) { return LinksBF16{c->Ubf, c->V}; }

void need_gauge(const dfl_ctx* c)
{
    if (!c->have_gauge)
        fail(DFL_ESTATE, "no gauge field: call dfl_set_gauge first");
}
void need_subspace(const dfl_ctx* c)
{
    if (!c->have_subspace)
        fail(DFL_ESTATE, "no deflation subspace: call dfl_setup first");
}
void need_ctx(const dfl_ctx* c)
{
    if (!c)
        fail(DFL_EINVAL, "null context");
}
void need_ptr(const void* p, const char* what)
{
    if (!p)
        fail(DFL_EINVAL, std::string("null pointer: ") + what);
}
void need_nrhs(const dfl_ctx* c, int nrhs)
{
    if (nrhs < 1 || nrhs > c->p.nrhs_max)
        fail(DFL_EINVAL, "nrhs must be in 1..nrhs_max");
}

void sync(dfl_ctx* c) { HIPCHECK(hipStreamSynchronize(c->stream)); }

// ------------------------------------------------------------- profiling

hipEvent_t prof_event(dfl_ctx* c)
{
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    HIPCHECK(hipEventCreate(&e));
    return e;
}

// records an event pair around the launches in its scope when profiling is on
struct ProfScope {
    dfl_ctx* c;
    int cls;
    hipEvent_t e0 = nullptr;
    ProfScope(dfl_ctx* cc, int k) : c(cc), cls(k)
    {
        if (c->prof_on && !c->capturing) {
            e0 = prof_event(c);
            HIPCHECK(hipEventRecord(e0, c->stream));
        }
    }
    ~ProfScope()
    {
        if (e0) {
            hipEvent_t e1 = prof_event(c);
            if (hipEventRecord(e1, c->stream) == hipSuccess)
                c->ev_pending.push_back({cls, {e0, e1}});
        }
    }
};

// fold recorded event pairs into the per-class sums (synchronises)
void prof_collect(dfl_ctx* c)
{
    if (c->ev_pending.empty())
        return;
    sync(c);
    for (auto& p : c->ev_pending) {
        float ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, p.second.first, p.second.second));
        c->prof_t[p.first] += ms * 1e-3;
        c->prof_n[p.first] += 1;
        c->ev_pool.push_back(p.second.first);
        c->ev_pool.push_back(p.second.second);
    }
    c->ev_pending.clear();
}

// copy the first n device scalars to the pinned host mirror and wait
void download(dfl_ctx* c, int n)
{
    HIPCHECK(hipMemcpyAsync(c->hscal, c->dscal, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    sync(c);
}

// the first n scalars of each of nb right-hand sides (stride S_TOTAL) to the host
void download_b(dfl_ctx* c, int n, int nb)
{
    HIPCHECK(hipMemcpy2DAsync(c->hscal, sizeof(double) * S_TOTAL, c->dscal, sizeof(double) * S_TOTAL,
                              sizeof(double) * n, nb, hipMemcpyDeviceToHost, c->stream));
    sync(c);
}

// per-RHS active mask to the device (host mirror is pinned; the previous copy
// has completed because every GCR step synchronises before the mask changes)
void upload_mask(dfl_ctx* c, const std::vector<int>& m)
{
    for (size_t b = 0; b < m.size(); ++b)
        c->hact[b] = m[b];
    HIPCHECK(hipMemcpyAsync(c->dact, c->hact, sizeof(int) * m.size(), hipMemcpyHostToDevice, c->stream));
}

// ||x_b||^2 of nb fields of n entries to the host (synchronises)
std::vector<double> host_norm2_b(dfl_ctx* c, const c64* x, long n, int nb)
{
    launch_norm2_b<double>(x, n, nb, n, c->red, c->dscal + S_R, S_TOTAL, nullptr, c->stream);
    HIPCHECK(hipMemcpy2DAsync(c->hscal + S_R, sizeof(double) * S_TOTAL, c->dscal + S_R, sizeof(double) * S_TOTAL,
                              sizeof(double), nb, hipMemcpyDeviceToHost, c->stream));
    sync(c);
    std::vector<double> out(nb);
    for (int b = 0; b < nb; ++b)
        out[b] = c->hscal[(long)b * S_TOTAL + S_R];
    return out;
}

// ||x||^2 to the host (synchronises)
template <typename T> double host_norm2(dfl_ctx* c, const cpx<T>* x, long n)
{
    launch_norm2<T>(x, n, c->red, c->dscal + S_R, c->stream);
    HIPCHECK(hipMemcpyAsync(c->hscal + S_R, c->dscal + S_R, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    sync(c);
    return c->hscal[S_R];
}

// ---------------------------------------------------------------- graphs

void drop_graphs(dfl_ctx* c)
{
    for (auto& g : c->graphs)
        (void)hipGraphExecDestroy(g.second);
    c->graphs.clear();
}

// Run body on the context's stream: directly, or (graphs on) as the replay of
// a graph captured from it the first time this key is seen. Capture and
// replay use the context's own stream gstream, ordered after the work already
// queued on `stream` and before the work queued after it by a pair of events,
// so the caller's stream may be any stream (the null stream included).
// Captured launch sequences must not contain memsets or host synchronisation.
void run_step(dfl_ctx* c, long key, const std::function<void()>& body)
{
    if (!c->use_graph) {
        body();
        return;
    }
    hipGraphExec_t exec = nullptr;
    for (auto& g : c->graphs)
        if (g.first == key)
            exec = g.second;
    HIPCHECK(hipEventRecord(c->gev[0], c->stream));
    HIPCHECK(hipStreamWaitEvent(c->gstream, c->gev[0], 0));
    if (!exec) {
        hipGraph_t graph = nullptr;
        hipStream_t user = c->stream;
        HIPCHECK(hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal));
        c->capturing = true;
        c->stream = c->gstream;
        try {
            body();
        } catch (...) {
            c->capturing = false;
            c->stream = user;
            (void)hipStreamEndCapture(c->gstream, &graph);
            if (graph)
                (void)hipGraphDestroy(graph);
            throw;
        }
        c->capturing = false;
        c->stream = user;
        HIPCHECK(hipStreamEndCapture(c->gstream, &graph));
        hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHECK(e);
        c->graphs.push_back({key, exec});
    }
    HIPCHECK(hipGraphLaunch(exec, c->gstream));
    HIPCHECK(hipEventRecord(c->gev[1], c->gstream));
    HIPCHECK(hipStreamWaitEvent(c->stream, c->gev[1], 0));
    ++c->graph_replays;
}

// ------------------------------------------------------------ operators

void dirac64(dfl_ctx* c, const c64* in, c64* out, double m0, int nb = 1)
{
    ProfScope ps(c, DFL_PROF_DIRAC);
    launch_dirac64(c->g, links64(c), in, out, nb, m0, 0, 0, 0, c->stream, c->Cl64);
}

// out = s - D in for nb fields (the subtraction fused into the stencil); out
// must alias neither s nor in
void dirac64_sub(dfl_ctx* c, const c64* s, const c64* in, c64* out, double m0, int nb = 1)
{
    ProfScope ps(c, DFL_PROF_DIRAC);
    launch_dirac64_sub(c->g, links64(c), s, in, out, nb, m0, c->stream, c->Cl64);
}

// psi = M_sap rho for nrhs fields (FP64 in and out; block solves in sap_prec).
// One launch per colour sweep covers all nrhs fields. rho_nrm2 (FP32 block
// solves only, may be null): rho_b enters divided by sqrt(rho_nrm2[2 b]), the
// scale applied while rho is rounded to FP32 (M_sap is linear). FP32 block
// solves leave the result in FP32 as well, in s32b or s32a: the pointer
// returned (null for FP64 block solves). rho32 (FP32 block solves, rho_nrm2
// required): rho is the FP32 result of an earlier call, s32a or s32b, which
// the sweeps read directly, scaled as they read it, writing into the other
// of the two (rho is then not read, and psi may be null: no FP64 result
// written). finite_flag (FP32 block solves with rho_nrm2 only): bit 1 set
// there if an entry of rho is not finite.
c32* sap_apply(dfl_ctx* c, const c64* rho, c64* psi, double m0, int nrhs = 1, const double* rho_nrm2 = nullptr,
               const c32* rho32 = nullptr, int* finite_flag = nullptr)
{
    const long n = c->field_elems * nrhs;
    const int ncy = c->p.ncy;
    // psi starts at zero: the first cycle's colour-0 sweep sees zero
    // everywhere, its colour-1 sweep zero on its own blocks (no fill pass)
    auto init_of = [](int cy, int col) { return cy > 0 ? 0 : (col == 0 ? 2 : 1); };
    if (c->p.sap_prec == DFL_F64) {
        for (int cy = 0; cy < ncy; ++cy)
            for (int col = 0; col < 2; ++col) {
                ProfScope ps(c, c->sap_prof_cls);
                launch_sap_colour64(c->g, c->sg, links64(c), rho, psi, m0, c->p.nmr, col, nrhs, init_of(cy, col),
                                    c->stream, c->Cl64);
            }
        return nullptr;
    }
    // FP32 block solves on FP32 copies; the last cycle's sweeps also write
    // their blocks' result to psi in FP64 (every block has one of the colours)
    const c32* in32 = c->s32a;
    c32* out32 = c->s32b;
    const double* scale_on_read = nullptr;
    if (rho32) {
        if (!rho_nrm2 || (rho32 != c->s32a && rho32 != c->s32b))
            fail(DFL_EINVAL, "Schwarz application: an FP32 input must be a staged result with its norms");
        in32 = rho32;
        out32 = rho32 == c->s32b ? c->s32a : c->s32b;
        scale_on_read = rho_nrm2;
    } else if (rho_nrm2)
        launch_f64_to_f32_scaled(rho, c->s32a, c->field_elems, nrhs, rho_nrm2, 2, c->stream, finite_flag);
    else
        launch_f64_to_f32(rho, c->s32a, n, c->stream);
    for (int cy = 0; cy < ncy; ++cy)
        for (int col = 0; col < 2; ++col) {
            ProfScope ps(c, c->sap_prof_cls);
            c64* out64 = cy == ncy - 1 ? psi : nullptr;
            if (c->p.link_prec == DFL_BF16)
                launch_sap_colour_bf16(c->g, c->sg, linksbf(c), in32, out32, (float)m0, c->p.nmr, col, nrhs,
                                       init_of(cy, col), out64, c->stream, c->Cl32, scale_on_read);
            else
                launch_sap_colour32(c->g, c->sg, links32(c), in32, out32, (float)m0, c->p.nmr, col, nrhs,
                                    init_of(cy, col), out64, c->stream, c->Cl32, scale_on_read);
        }
    return out32;
}

// ------------------------------------------------------------------ GCR
//
// Flexible restarted GCR (section 6.2) for nb right-hand sides in lockstep:
// xi_k = M rho, chi_k = Op xi_k, orthogonalised against chi_{<k} (classical
// Gram-Schmidt, a second pass where the first cancelled more than 99% of
// ||chi_k||^2), normalised, rho -= (chi_k, rho) chi_k. Every
// step is one batched launch sequence over all sources; each source has its
// own coefficients and leaves the cycle when it converges. At the end of a
// cycle the coefficients alpha solve the triangular system, x += sum alpha_k
// xi_k and the residue is recomputed from scratch (appendix A.5).
//
// Layout: residue and solution of source b at b*n; Krylov slot k of source b
// at (k*nb + b)*n. Scalars of source b at dscal + b*S_TOTAL.

struct GcrVecs {
    c64* xi;   // nkv * nb vectors
    c64* chi;  // nkv * nb vectors
    c64* r;    // nb residues
    c64* x;    // nb solution accumulators
};

struct GcrResult {
    int status;
    int iters;
    int restarts;
    double rel;  // last recomputed relative residual
};

using BatchOp = std::function<void(const c64*, c64*, int)>;

// inner_tol(ratio) gives the relative tolerance of the inner little solves
// for the step when the residues have fallen by `ratio` (the smallest
// rho_k / rho_cycle-start over the sources still in the cycle) within the
// cycle; it is written to c->dtol before the step runs.
std::vector<GcrResult> gcr_run(dfl_ctx* c, long n, int nb, int nkv, int maxiter, double tol,
                               const std::vector<double>& src_norm, GcrVecs v, const BatchOp& precond,
                               const BatchOp& op, const BatchOp& recompute_residual, double cycle_floor = 0.0,
                               std::vector<double>* history_ = nullptr,
                               const std::function<double(double)>& inner_tol = nullptr)
{
    std::vector<GcrResult> res(nb, GcrResult{DFL_OK, 0, 0, 0.0});
    launch_zero<double>(v.x, n * nb, c->stream);
    // the caller has put the initial residues in r
    std::vector<double> rn = host_norm2_b(c, v.r, n, nb);
    for (auto& q : rn)
        q = std::sqrt(q);
    if (history_)
        history_->push_back(src_norm[0] > 0.0 ? rn[0] / src_norm[0] : 0.0);
    std::vector<int> done(nb, 0), act(nb, 0), kb(nb, 0);
    std::vector<cd> a((size_t)nb * nkv * nkv), cc((size_t)nb * nkv), alpha((size_t)nb * nkv);
    std::vector<double> bb((size_t)nb * nkv), rn_cycle(nb);
    const long ks = n * nb;  // stride of the Krylov slots
    const int* mask = nb > 1 ? c->dact : nullptr;
    while (true) {
        int n_act = 0;
        for (int b = 0; b < nb; ++b) {
            if (done[b])
                continue;
            res[b].rel = src_norm[b] > 0.0 ? rn[b] / src_norm[b] : 0.0;
            if (!std::isfinite(rn[b]))
                fail(DFL_ENONFINITE, "non-finite residual in GCR");
            if (src_norm[b] == 0.0 || rn[b] <= tol * src_norm[b]) {
                done[b] = 1;
            } else if (res[b].iters >= maxiter) {
                res[b].status = DFL_NOT_CONVERGED;
                done[b] = 1;
            }
        }
        for (int b = 0; b < nb; ++b) {
            act[b] = !done[b];
            kb[b] = 0;
            rn_cycle[b] = rn[b];
            n_act += act[b];
        }
        if (n_act == 0)
            return res;
        if (mask)
            upload_mask(c, act);
        int k = 0;
        while (k < nkv && n_act > 0) {
            c64* xk = v.xi + (long)k * ks;
            c64* ck = v.chi + (long)k * ks;
            if (inner_tol) {
                double ratio = 1.0;
                for (int b = 0; b < nb; ++b)
                    if (act[b] && rn_cycle[b] > 0.0)
                        ratio = std::min(ratio, rn[b] / rn_cycle[b]);
                *c->htol = inner_tol(ratio);
                HIPCHECK(hipMemcpyAsync(c->dtol, c->htol, sizeof(double), hipMemcpyHostToDevice, c->stream));
            }
            run_step(c, (long)k * 64 + nb, [&]() {
                precond(v.r, xk, nb);
                op(xk, ck, nb);
                if (k > 0) {
                    // classical Gram-Schmidt; the first pass also yields ||chi_k||^2 (slot k, as chi_k
                    // follows the earlier images at stride ks), and a second pass runs only for the
                    // sources whose first pass cancelled more than 99% of it
                    launch_multidot_b<double>(v.chi, ks, k + 1, ck, n, nb, n, n, c->red, c->dscal + S_A1, S_TOTAL,
                                              mask, c->stream);
                    launch_multiaxpy_b<double>(v.chi, ks, k, c->dscal + S_A1, S_TOTAL, -1.0, ck, n, nb, n, n, mask,
                                               c->stream);
                    launch_second_pass_mask(c->dscal + S_A1, c->dscal + S_A2, k, S_TOTAL, mask, nb, c->dact2,
                                            c->stream);
                    launch_multidot_b<double>(v.chi, ks, k, ck, n, nb, n, n, c->red, c->dscal + S_A2, S_TOTAL,
                                              c->dact2, c->stream);
                    launch_multiaxpy_b<double>(v.chi, ks, k, c->dscal + S_A2, S_TOTAL, -1.0, ck, n, nb, n, n,
                                               c->dact2, c->stream);
                }
                // ||chi||^2 and (chi, r) in one pass (S_B, S_C), then chi /= ||chi||,
                // r -= ((chi, r) / ||chi||^2) chi and ||r||^2 (S_R) in another
                static_assert(S_C == S_B + 2, "the norm and the product are reduced together");
                launch_norm_dot_b(ck, v.r, n, nb, n, c->red, c->dscal + S_B, S_TOTAL, mask, c->stream);
                launch_scale_update_b(ck, v.r, n, nb, n, c->dscal + S_B, S_TOTAL, c->red, c->dscal + S_R, S_TOTAL,
                                      mask, c->stream);
            });
            download_b(c, S_DOWN, nb);
            bool changed = false;
            for (int b = 0; b < nb; ++b) {
                if (!act[b])
                    continue;
                const double* h = c->hscal + (long)b * S_TOTAL;
                cd* ab = &a[(size_t)b * nkv * nkv];
                for (int j = 0; j < k; ++j)
                    ab[(size_t)j * nkv + k] = cd(h[S_A1 + 2 * j] + h[S_A2 + 2 * j], h[S_A1 + 2 * j + 1] + h[S_A2 + 2 * j + 1]);
                const double bk = std::sqrt(h[S_B]);
                bb[(size_t)b * nkv + k] = bk;
                // (chi_k, r) for the unit chi_k: S_C holds the product before the scaling
                cc[(size_t)b * nkv + k] = bk > 0.0 ? cd(h[S_C], h[S_C + 1]) / bk : cd(0.0, 0.0);
                rn[b] = std::sqrt(h[S_R]);
                if (!(bk > 0.0) || !std::isfinite(bk))
                    fail(bk == 0.0 ? DFL_ESINGULAR : DFL_ENONFINITE, "GCR breakdown: zero or non-finite Krylov image");
                kb[b] = k + 1;
                ++res[b].iters;
                if (history_ && b == 0)
                    history_->push_back(rn[0] / src_norm[0]);
                if (rn[b] <= tol * src_norm[b] || rn[b] <= cycle_floor * rn_cycle[b] || res[b].iters >= maxiter) {
                    act[b] = 0;
                    --n_act;
                    changed = true;
                }
            }
            ++k;
            if (changed && mask && n_act > 0 && k < nkv)
                upload_mask(c, act);
        }
        int kmax = 0;
        for (int b = 0; b < nb; ++b) {
            const cd* ab = &a[(size_t)b * nkv * nkv];
            cd* al = &alpha[(size_t)b * nkv];
            for (int i = kb[b] - 1; i >= 0; --i) {
                cd t = cc[(size_t)b * nkv + i];
                for (int j = i + 1; j < kb[b]; ++j)
                    t -= ab[(size_t)i * nkv + j] * al[j];
                al[i] = t / bb[(size_t)b * nkv + i];
            }
            double* up = c->hscal + (long)b * S_TOTAL + S_ALPHA;
            for (int i = 0; i < nkv; ++i) {
                up[2 * i] = i < kb[b] ? al[i].real() : 0.0;
                up[2 * i + 1] = i < kb[b] ? al[i].imag() : 0.0;
            }
            kmax = std::max(kmax, kb[b]);
            act[b] = kb[b] > 0;
        }
        HIPCHECK(hipMemcpy2DAsync(c->dscal + S_ALPHA, sizeof(double) * S_TOTAL, c->hscal + S_ALPHA,
                                  sizeof(double) * S_TOTAL, sizeof(double) * 2 * nkv, nb, hipMemcpyHostToDevice,
                                  c->stream));
        if (mask)
            upload_mask(c, act);
        launch_multiaxpy_b<double>(v.xi, ks, kmax, c->dscal + S_ALPHA, S_TOTAL, 1.0, v.x, n, nb, n, n, mask,
                                   c->stream);
        recompute_residual(v.x, v.r, nb);
        rn = host_norm2_b(c, v.r, n, nb);
        for (int b = 0; b < nb; ++b) {
            rn[b] = std::sqrt(rn[b]);
            if (kb[b] > 0)
                ++res[b].restarts;
            if (done[b])
                res[b].rel = src_norm[b] > 0.0 ? rn[b] / src_norm[b] : 0.0;
        }
    }
}

// ---------------------------------------------------------- little solve

// v_b = A^{-1} w_b to ||w_b - A v_b|| <= tol ||w_b|| (eq. (6.1)) for nb little
// vectors back to back; FP64 in and out. One cooperative launch; iteration
// counts accumulate in c->lstats.
void little_solve_impl(dfl_ctx* c, const c64* w, c64* v, double tol, dfl_prec prec, int nb = 1,
                       const double* tol_dev = nullptr)
{
    const long n = (long)c->g.Nb * c->p.Ns;
    const int Ns = c->p.Ns, nkv = c->p.little_nkv, mi = c->p.little_maxiter;
    const bool eo_multi = nb > 1 && c->eo_ok && little_eo_fits(c->g, c->lgrid_multi);
    if (prec == DFL_F64) {
        ProfScope ps(c, DFL_PROF_LITTLE);
        if (nb == 1)
            launch_little_gcr<double>(c->g, Ns, nkv, mi, tol, tol_dev, c->At64, c->eo_ok ? c->Mt64 : nullptr,
                                      static_cast<c64*>(c->lw1), static_cast<c64*>(c->lw2), c->gQ, c->gZ,
                                      c->eo_ok ? c->gdefl_n : 0, c->gdefl_oblique, c->gAinv, c->gGw, w, v,
                                      static_cast<c64*>(c->lr),
                                      static_cast<c64*>(c->lxi), static_cast<c64*>(c->lchi), c->lpart, c->lstats,
                                      c->lbar_count, c->lbar_gen, c->lgrid, c->stream, !c->capturing);
        else
            launch_little_gcr_multi<double>(c->g, Ns, nkv, mi, tol, tol_dev, nb, c->At64, eo_multi ? c->Mt64 : nullptr,
                                            static_cast<c64*>(c->lw1), static_cast<c64*>(c->lw2), w, v,
                                            static_cast<c64*>(c->lr),
                                            static_cast<c64*>(c->lxi), static_cast<c64*>(c->lchi), c->lpart, c->lfin,
                                            c->lacoef, c->lstats, c->lbar_count, c->lbar_gen,
                                            c->lgrid_multi, c->stream, !c->capturing);
    } else {
        launch_f64_to_f32(w, c->lw32, n * nb, c->stream);
        {
            ProfScope ps(c, DFL_PROF_LITTLE);
            if (nb == 1)
                launch_little_gcr<float>(c->g, Ns, nkv, mi, tol, tol_dev, c->At32, c->eo_ok ? c->Mt32 : nullptr,
                                         static_cast<c32*>(c->lw1), static_cast<c32*>(c->lw2), c->gQ32, c->gZ32,
                                         c->eo_ok ? c->gdefl_n : 0, c->gdefl_oblique, c->gAinv, c->gGw, c->lw32,
                                         c->lx32, static_cast<c32*>(c->lr),
                                         static_cast<c32*>(c->lxi), static_cast<c32*>(c->lchi), c->lpart, c->lstats,
                                         c->lbar_count, c->lbar_gen, c->lgrid, c->stream, !c->capturing);
            else
                launch_little_gcr_multi<float>(c->g, Ns, nkv, mi, tol, tol_dev, nb, c->At32,
                                               eo_multi ? c->Mt32 : nullptr, static_cast<c32*>(c->lw1),
                                               static_cast<c32*>(c->lw2), c->lw32, c->lx32,
                                               static_cast<c32*>(c->lr), static_cast<c32*>(c->lxi),
                                               static_cast<c32*>(c->lchi), c->lpart, c->lfin, c->lacoef, c->lstats,
                                               c->lbar_count, c->lbar_gen, c->lgrid_multi, c->stream, !c->capturing);
        }
        launch_f32_to_f64(c->lx32, v, n * nb, c->stream);
    }
}

void reset_little_stats(dfl_ctx* c) { HIPCHECK(hipMemsetAsync(c->lstats, 0, sizeof(int) * 4, c->stream)); }

// [iterations, solves, failed] accumulated since the last reset (synchronises)
void read_little_stats(dfl_ctx* c, int out[3])
{
    int h[4];
    HIPCHECK(hipMemcpyAsync(h, c->lstats, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    sync(c);
    out[0] = h[0];
    out[1] = h[1];
    out[2] = h[2] & 1;
    if (c->prof_on)
        c->prof_little_iters += h[0];
    if (h[2] & 4) {
        // a timed-out barrier leaves its arrival count behind: clear it so
        // that later solves start from a clean barrier
        HIPCHECK(hipMemsetAsync(c->lbar_count, 0, sizeof(unsigned) * 64, c->stream));
        HIPCHECK(hipMemsetAsync(c->lstats, 0, sizeof(int) * 4, c->stream));
        sync(c);
        fail(DFL_EHIP, "little solver: grid barrier timed out");
    }
}

// out = Phi A^{-1} Phi^+ in  (eq. (3.10)'s coarse term) for nb fields; out may not alias in.
// Inexact (FP32) inner projections read the FP32 copy of the basis.
void coarse(dfl_ctx* c, const c64* in, c64* out, double tol, dfl_prec prec, int nb = 1,
            const double* tol_dev = nullptr)
{
    c64* w = static_cast<c64*>(c->lw);
    c64* x = static_cast<c64*>(c->lx);
    const bool b32 = prec == DFL_F32 && c->Phi32;
    {
        ProfScope ps(c, DFL_PROF_PROJECT);
        if (b32)
            launch_restrict_b32(c->g, c->Phi32, c->p.Ns, in, w, nb, c->stream);
        else
            launch_restrict64(c->g, c->Phi, c->p.Ns, in, w, nb, c->stream);
    }
    little_solve_impl(c, w, x, tol, prec, nb, tol_dev);
    ProfScope ps(c, DFL_PROF_PROJECT);
    if (b32)
        launch_prolong_b32(c->g, c->Phi32, c->p.Ns, x, out, nb, c->stream);
    else
        launch_prolong64(c->g, c->Phi, c->p.Ns, x, out, nb, c->stream);
}

// out = P_L in = in - D coarse(in)   (eq. (3.3)) for nb fields
void apply_PL(dfl_ctx* c, const c64* in, c64* out, double tol, dfl_prec prec, c64* tmpA, c64* tmpB, int nb = 1,
              const double* tol_dev = nullptr)
{
    coarse(c, in, tmpA, tol, prec, nb, tol_dev);
    if (out != in) {
        dirac64_sub(c, in, tmpA, out, c->p.m0, nb);
    } else {
        dirac64(c, tmpA, tmpB, c->p.m0, nb);
        launch_sub<double>(in, tmpB, out, c->field_elems * nb, c->stream);
    }
}

// Even-odd matrices of the little operator (appendix A.2) after A changed;
// the plain system is kept if a diagonal block is not safely invertible or
// the block lists do not fit. Synchronises.
void prepare_eo(dfl_ctx* c)
{
    c->eo_ok = false;
    if (!c->p.little_eo || !c->Mt64 || !little_eo_fits(c->g, c->lgrid))
        return;
    HIPCHECK(hipMemsetAsync(c->dflag + 1, 0, sizeof(int), c->stream));
    launch_little_eo_prep(c->g, c->A64, c->p.Ns, c->Mt64, c->Mt32, c->dflag + 1, c->stream);
    HIPCHECK(hipGetLastError());
    int f = 0;
    HIPCHECK(hipMemcpyAsync(&f, c->dflag + 1, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    sync(c);
    c->eo_ok = (f & 1) == 0;
}

// Global-mode deflation of the even-odd little system (appendix A.3): the
// start fields in the block basis on even blocks, u_l, their images
// W = A_hat U, and Q = W C, Z = U C with C from Cholesky-QR applied twice so
// that Q is orthonormal and Q = A_hat Z. The little GCR then keeps its
// residue orthogonal to span Q. Off (gdefl_n = 0) if the even-odd system is
// off or W is numerically rank deficient. Synchronises.
// G = R^H R with R upper triangular, computed for the leading n' <= n columns
// whose pivots stay above 1e-12 of the largest diagonal entry (the later
// columns are numerically dependent on them). On return G holds R^-1 for
// those n' columns, zero elsewhere; returns n'.
int cholesky_inverse(std::vector<cd>& G, int n)
{
    std::vector<cd> R((size_t)n * n, cd(0.0, 0.0));
    double scale = 0.0;
    for (int i = 0; i < n; ++i)
        scale = std::max(scale, G[(size_t)i * n + i].real());
    int m = 0;
    for (int j = 0; j < n; ++j) {
        double d = G[(size_t)j * n + j].real();
        for (int k = 0; k < j; ++k)
            d -= std::norm(R[(size_t)k * n + j]);
        if (!(d > 1e-12 * scale))
            break;
        const double rjj = std::sqrt(d);
        R[(size_t)j * n + j] = rjj;
        for (int i = j + 1; i < n; ++i) {
            cd t = G[(size_t)j * n + i];
            for (int k = 0; k < j; ++k)
                t -= std::conj(R[(size_t)k * n + j]) * R[(size_t)k * n + i];
            R[(size_t)j * n + i] = t / rjj;
        }
        m = j + 1;
    }
    std::vector<cd> Inv((size_t)n * n, cd(0.0, 0.0));
    for (int col = 0; col < m; ++col)
        for (int i = col; i >= 0; --i) {
            cd t = (i == col) ? cd(1.0, 0.0) : cd(0.0, 0.0);
            for (int k = i + 1; k <= col; ++k)
                t -= R[(size_t)i * n + k] * Inv[(size_t)k * n + col];
            Inv[(size_t)i * n + col] = t / R[(size_t)i * n + i];
        }
    G = Inv;
    return m;
}

// Dense inverse of an n x n complex matrix (row-major) by Gauss-Jordan with
// partial pivoting; false if a pivot falls below 1e-12 of the largest entry.
bool invert_dense(std::vector<cd>& M, int n)
{
    std::vector<cd> I((size_t)n * n, cd(0.0, 0.0));
    for (int i = 0; i < n; ++i)
        I[(size_t)i * n + i] = 1.0;
    double big = 0.0;
    for (const cd& z : M)
        big = std::max(big, std::abs(z));
    if (!(big > 0.0))
        return false;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::abs(M[(size_t)r * n + col]) > std::abs(M[(size_t)piv * n + col]))
                piv = r;
        if (!(std::abs(M[(size_t)piv * n + col]) > 1e-12 * big))
            return false;
        if (piv != col)
            for (int j = 0; j < n; ++j) {
                std::swap(M[(size_t)piv * n + j], M[(size_t)col * n + j]);
                std::swap(I[(size_t)piv * n + j], I[(size_t)col * n + j]);
            }
        const cd inv = 1.0 / M[(size_t)col * n + col];
        for (int j = 0; j < n; ++j) {
            M[(size_t)col * n + j] *= inv;
            I[(size_t)col * n + j] *= inv;
        }
        for (int r = 0; r < n; ++r) {
            if (r == col)
                continue;
            const cd f = M[(size_t)r * n + col];
            if (f == cd(0.0, 0.0))
                continue;
            for (int j = 0; j < n; ++j) {
                M[(size_t)r * n + j] -= f * M[(size_t)col * n + j];
                I[(size_t)r * n + j] -= f * I[(size_t)col * n + j];
            }
        }
    }
    M = I;
    return true;
}

// Section 3's projectors on the even-odd little system (appendix A.3 as the
// paper states it): Z = the even-block global modes, orthonormalised
// (Cholesky-QR twice), W = A_hat Z, the "little little" operator Z^+ W
// inverted exactly on the host; the little GCR then applies
// P_L = 1 - W (Z^+ W)^-1 Z^+ to every new Krylov image and to the residue at
// the start and at every restart, and the solution picks up Z (Z^+ W)^-1 Z^+
// of the residue. Synchronises; off (gdefl_n = 0) if Z^+ W is not safely
// invertible.
void prepare_gdefl_oblique(dfl_ctx* c)
{
    const int Ns = c->p.Ns;
    const long N = (long)c->g.Nb * Ns;
    launch_global_modes(c->g, c->gsR, Ns, c->gU, c->stream);
    std::vector<cd> G;
    int nq = Ns;
    for (int pass = 0; pass < 2; ++pass) {
        c64* X = pass == 0 ? c->gU : c->gZ;
        c64* Xout = pass == 0 ? c->gZ : c->gU;
        launch_gram(X, N, nq, c->gC, c->stream);
        G.assign((size_t)nq * nq, cd(0.0, 0.0));
        HIPCHECK(hipMemcpyAsync(G.data(), c->gC, sizeof(c64) * nq * nq, hipMemcpyDeviceToHost, c->stream));
        sync(c);
        const int m = cholesky_inverse(G, nq);
        if (m == 0)
            return;
        std::vector<cd> C((size_t)nq * m);
        for (int k = 0; k < nq; ++k)
            for (int l = 0; l < m; ++l)
                C[(size_t)k * m + l] = G[(size_t)k * nq + l];
        HIPCHECK(hipMemcpyAsync(c->gC, C.data(), sizeof(c64) * nq * m, hipMemcpyHostToDevice, c->stream));
        launch_combine(X, N, nq, m, c->gC, Xout, c->stream);
        sync(c);
        nq = m;
    }
    std::swap(c->gZ, c->gU);  // Z (orthonormal, nq columns) now in gZ
    // W = A_hat Z on the even blocks: odd = M_oe Z, then even = Z - M_eo (odd)
    launch_zero<double>(c->gW, N * Ns, c->stream);
    launch_zero<double>(c->gQ, N * Ns, c->stream);
    launch_eo_hop(c->g, c->Mt64, Ns, c->gZ, nullptr, c->gW, nq, 1, 0.0, 1.0, c->stream);
    launch_eo_hop(c->g, c->Mt64, Ns, c->gW, c->gZ, c->gQ, nq, 0, 1.0, -1.0, c->stream);
    std::vector<cd> Ac((size_t)nq * nq), Gw((size_t)nq * nq);
    launch_gram2(c->gZ, c->gQ, N, nq, c->gC, c->stream);
    HIPCHECK(hipMemcpyAsync(Ac.data(), c->gC, sizeof(c64) * nq * nq, hipMemcpyDeviceToHost, c->stream));
    sync(c);
    launch_gram(c->gQ, N, nq, c->gC, c->stream);
    HIPCHECK(hipMemcpyAsync(Gw.data(), c->gC, sizeof(c64) * nq * nq, hipMemcpyDeviceToHost, c->stream));
    sync(c);
    if (!invert_dense(Ac, nq))
        return;
    HIPCHECK(hipMemcpyAsync(c->gAinv, Ac.data(), sizeof(c64) * nq * nq, hipMemcpyHostToDevice, c->stream));
    HIPCHECK(hipMemcpyAsync(c->gGw, Gw.data(), sizeof(c64) * nq * nq, hipMemcpyHostToDevice, c->stream));
    launch_c64_to_c32(c->gQ, c->gQ32, N * Ns, c->stream);
    launch_c64_to_c32(c->gZ, c->gZ32, N * Ns, c->stream);
    HIPCHECK(hipGetLastError());
    sync(c);  // Ac and Gw are host memory read by the copies
    c->gdefl_n = nq;
    c->gdefl_oblique = true;
}

void prepare_gdefl(dfl_ctx* c)
{
    c->gdefl_n = 0;
    c->gdefl_oblique = false;
    if (!c->p.little_gdefl || !c->eo_ok || !c->gU)
        return;
    if (c->p.little_gdefl == 2) {
        prepare_gdefl_oblique(c);
        return;
    }
    const int Ns = c->p.Ns;
    const long N = (long)c->g.Nb * Ns;
    launch_global_modes(c->g, c->gsR, Ns, c->gU, c->stream);
    launch_zero<double>(c->gW, N * Ns, c->stream);
    launch_zero<double>(c->gQ, N * Ns, c->stream);
    launch_eo_hop(c->g, c->Mt64, Ns, c->gU, nullptr, c->gQ, Ns, 1, 0.0, 1.0, c->stream);  // odd: M_oe u
    launch_eo_hop(c->g, c->Mt64, Ns, c->gQ, c->gU, c->gW, Ns, 0, 1.0, -1.0, c->stream);   // even: u - M_eo (M_oe u)
    std::vector<cd> G((size_t)Ns * Ns);
    int nq = Ns;
    for (int pass = 0; pass < 2; ++pass) {
        c64* X = pass == 0 ? c->gW : c->gQ;
        c64* Zin = pass == 0 ? c->gU : c->gZ;
        c64* Xout = pass == 0 ? c->gQ : c->gW;
        c64* Zout = pass == 0 ? c->gZ : c->gU;
        launch_gram(X, N, nq, c->gC, c->stream);
        G.assign((size_t)nq * nq, cd(0.0, 0.0));
        HIPCHECK(hipMemcpyAsync(G.data(), c->gC, sizeof(c64) * nq * nq, hipMemcpyDeviceToHost, c->stream));
        sync(c);
        const int m = cholesky_inverse(G, nq);
        if (m == 0)
            return;
        // keep the leading m directions: C is nq x m (the first m columns of R^-1)
        std::vector<cd> C((size_t)nq * m);
        for (int k = 0; k < nq; ++k)
            for (int l = 0; l < m; ++l)
                C[(size_t)k * m + l] = G[(size_t)k * nq + l];
        HIPCHECK(hipMemcpyAsync(c->gC, C.data(), sizeof(c64) * nq * m, hipMemcpyHostToDevice, c->stream));
        launch_combine(X, N, nq, m, c->gC, Xout, c->stream);
        launch_combine(Zin, N, nq, m, c->gC, Zout, c->stream);
        sync(c);  // C is host memory read by the copy
        nq = m;
    }
    // after two passes Q, Z sit in gW, gU: swap the roles
    std::swap(c->gQ, c->gW);
    std::swap(c->gZ, c->gU);
    // accept only an orthonormal Q
    launch_gram(c->gQ, N, nq, c->gC, c->stream);
    G.assign((size_t)nq * nq, cd(0.0, 0.0));
    HIPCHECK(hipMemcpyAsync(G.data(), c->gC, sizeof(c64) * nq * nq, hipMemcpyDeviceToHost, c->stream));
    sync(c);
    for (int k = 0; k < nq; ++k)
        for (int l = 0; l < nq; ++l)
            if (std::abs(G[(size_t)k * nq + l] - cd(k == l ? 1.0 : 0.0, 0.0)) > 1e-8)
                return;
    launch_c64_to_c32(c->gQ, c->gQ32, N * Ns, c->stream);
    launch_c64_to_c32(c->gZ, c->gZ32, N * Ns, c->stream);
    HIPCHECK(hipGetLastError());
    c->gdefl_n = nq;
}

// Relaxed inverse iteration of eq. (5.1) on n native FP64 fields: from the
// fields at src (read only) into dst (src == dst: in place), normalise, then
// `steps` times psi <- M_sap psi at m0_setup and normalise. With
// normalise_out false the last normalisation is left out (for callers that
// only use the span of each field, e.g. the block Gram-Schmidt of the
// subspace setup, which is invariant under positive scale factors).
// Sets c->dflag bit 0 on non-finite input.
void inverse_iterate(dfl_ctx* c, const c64* src, c64* dst, int n, int steps, bool normalise_out = true)
{
    const long F = c->field_elems;
    // the n fields (back to back) are checked and normalised one launch per kernel
    auto normalise = [&]() {
        // a reduction writes a complex pair per field: stride 2
        launch_norm2_b<double>(dst, F, n, F, c->red, c->dnorm, 2, nullptr, c->stream);
        launch_scale_invsqrt_b<double>(dst, F, n, F, c->dnorm, 2, nullptr, c->stream);
    };
    const bool fp32 = c->p.sap_prec != DFL_F64 && steps > 0;
    // (the FP32 path checks src while its first step rounds it to FP32)
    if (!fp32)
        launch_finite_check<double>(src, F * n, c->dflag, c->stream);
    // the sweeps of the inverse iteration are timed as setup work
    struct SetupSweeps {
        dfl_ctx* c;
        explicit SetupSweeps(dfl_ctx* cc) : c(cc) { c->sap_prof_cls = DFL_PROF_SETUP_SAP; }
        ~SetupSweeps() { c->sap_prof_cls = DFL_PROF_SAP; }
    } setup_sweeps(c);
    if (!fp32) {
        if (src != dst)
            HIPCHECK(hipMemcpyAsync(dst, src, sizeof(c64) * F * n, hipMemcpyDeviceToDevice, c->stream));
        for (int step = 0; step < steps; ++step) {
            normalise();
            sap_apply(c, dst, c->tN, c->p.m0_setup, n);
            launch_copy<double>(c->tN, dst, F * n, c->stream);
        }
        if (normalise_out || steps == 0)
            normalise();
        return;
    }
    // FP32 block solves: each normalisation before a step is the scale of the
    // step's input (M_sap is linear, so the step maps the normalised field).
    // The first step rounds src to FP32 with that scale; the later ones read
    // the previous step's FP32 result in place, scaling it as the sweeps read
    // it, and write into the other FP32 buffer. Only the last step writes dst
    // in FP64; a final normalisation rewrites the fields
    const c32* cur = nullptr;
    for (int step = 0; step < steps; ++step) {
        const bool last = step == steps - 1;
        if (step == 0)
            launch_norm2_b<double>(src, F, n, F, c->red, c->dnorm, 2, nullptr, c->stream);
        else
            launch_norm2_b<float>(cur, F, n, F, c->red, c->dnorm, 2, nullptr, c->stream);
        cur = sap_apply(c, src, last ? dst : nullptr, c->p.m0_setup, n, c->dnorm, cur,
                        step == 0 ? c->dflag : nullptr);
    }
    if (normalise_out)
        normalise();
}

int max_multi_fields(const dfl_ctx* c)
{
    return c->p.sap_prec == DFL_F64 ? c->p.Ns : std::max(c->p.Ns, c->p.nrhs_max);
}

template <typename T> T* grow(dfl_ctx* c, T* p, size_t& have, size_t need)
{
    if (need <= have)
        return p;
    sync(c);
    if (p)
        HIPCHECK(hipFree(p));
    have = 0;
    T* q = alloc_dev<T>(c, need);
    have = need;
    return q;
}

// Block Gram-Schmidt (eq. (4.2)) of the Ns fields at src into Phi and the
// little operator (eq. (A.1)) at mass mA, with the even-odd and global-mode
// preparation. Synchronises; fails on non-finite fields or rank loss.
void build_subspace(dfl_ctx* c, const c64* src, double mA)
{
    const long F = c->field_elems;
    const int Ns = c->p.Ns;
    if (src != c->Phi)
        HIPCHECK(hipMemcpyAsync(c->Phi, src, sizeof(c64) * F * Ns, hipMemcpyDeviceToDevice, c->stream));
    ProfScope ps_setup(c, DFL_PROF_SETUP);
    // little operator, eq. (A.1): block-diagonal part and the eight face
    // hops, applied to a chunk of basis fields per launch (the Krylov
    // buffer is free during the setup), then the block products with Phi.
    // Chunk of basis fields per launch: bounded by the Krylov buffer (the
    // stencil output) and by t1 (the split partial sums, Nb*Ns*chunk entries)
    const long part_cap = F * c->p.nrhs_max;
    const long kcap = (long)c->p.nkv * c->p.nrhs_max;  // fields of each Krylov buffer
    const int chunk = (int)std::max(1L, std::min({(long)Ns, (long)little_columns_max(Ns), kcap, (long)(128 - Ns),
                                                  part_cap / ((long)c->g.Nb * Ns)}));
    // All Ns columns of a direction in one matrix-core launch when the two
    // Krylov buffers hold them (each basis block then read once per direction)
    const bool all = little_columns_all_ok(Ns, part_cap, c->g.Nb) && Ns <= 2 * kcap;
    // The faces along x2 and x3 are scattered in the native in-block order
    // (x3 fastest); their hops and block products read a copy of the basis in
    // the transposed order, where those faces are whole tiles or long runs.
    const bool tl = all || little_columns_transposable(Ns, chunk);
    if (tl)
        c->PhiT = grow<c64>(c, c->PhiT, c->PhiT_n, (size_t)F * Ns);
    // block Gram-Schmidt (eq. (4.2)); the 256-site block kernel also writes the
    // transposed copy and the FP32 copy of the basis
    const bool copies = launch_block_gs64(c->g, c->Phi, Ns, 1e-10, c->dflag, c->gsR, c->stream,
                                          tl ? c->PhiT : nullptr, c->Phi32);
    if (tl && !copies)
        launch_to_transposed(c->g, c->Phi, c->PhiT, Ns, c->stream);
    for (int d = 0; all && d < 9; ++d) {
        const int mu = d == 0 ? -1 : (d - 1) / 2;
        const bool t = mu >= 2;
        const c64* basis = t ? c->PhiT : c->Phi;
        const int n1 = (int)std::min<long>(Ns, kcap);
        for (int h = 0; h < 2; ++h) {
            const int l0 = h == 0 ? 0 : n1, nc = h == 0 ? n1 : Ns - n1;
            c64* y = h == 0 ? c->xi : c->chi;
            if (nc == 0)
                continue;
            if (d == 0)
                launch_dirac64(c->g, links64(c), basis + (long)l0 * F, y, nc, mA, 1, 0, 0, c->stream, c->Cl64);
            else
                launch_dirac64_face(c->g, links64(c), basis + (long)l0 * F, y, nc, mu, (d & 1) ? +1 : -1, c->stream,
                                    t);
        }
        launch_little_columns64_all(c->g, basis, Ns, c->xi, n1, c->chi, d, c->A64, c->t1, part_cap, c->stream, t);
    }
    for (int l0 = 0; !all && l0 < Ns; l0 += chunk) {
        const int nc = std::min(chunk, Ns - l0);
        for (int d = 0; d < 9; ++d) {
            const int mu = d == 0 ? -1 : (d - 1) / 2;
            const bool t = tl && mu >= 2;
            const c64* basis = t ? c->PhiT : c->Phi;
            const c64* f = basis + (long)l0 * F;
            if (d == 0)
                launch_dirac64(c->g, links64(c), f, c->xi, nc, mA, 1, 0, 0, c->stream, c->Cl64);
            else
                launch_dirac64_face(c->g, links64(c), f, c->xi, nc, mu, (d & 1) ? +1 : -1, c->stream, t);
            launch_little_columns64(c->g, basis, Ns, c->xi, nc, l0, d, c->A64, c->t1, part_cap, c->stream, t);
        }
    }
    launch_little_copies(c->A64, c->A32, c->At64, c->At32, (long)c->g.Nb * 9, Ns, c->stream);
    if (c->Phi32 && !copies)
        launch_f64_to_f32(c->Phi, c->Phi32, F * Ns, c->stream);
    c->eo_ok = false;
    c->m0_A = mA;
    int flag[4];
    HIPCHECK(hipMemcpyAsync(flag, c->dflag, sizeof(flag), hipMemcpyDeviceToHost, c->stream));
    sync(c);
    if (flag[0] & 1)
        fail(DFL_ENONFINITE, "non-finite entries in the start fields");
    if (flag[0] & 2)
        fail(DFL_ESINGULAR, "block Gram-Schmidt lost rank: the start fields are linearly dependent on a block");
    prepare_eo(c);
    prepare_gdefl(c);
}

// One bootstrapped inverse-iteration step (section 5.3) on the Ns fields f,
// with the subspace current in the context (built from f at m0_setup): each
// field psi becomes P_R chi + Phi A^-1 Phi^+ psi (eq. (3.10)) with chi = M_sap
// P_L psi, the approximate solution of the deflated equation P_L D chi =
// P_L psi (eq. (3.11)) after its preconditioner, and is normalised. Little
// solves to little_tol_in in little_prec; the Schwarz procedure runs on all
// fields in one launch per sweep.
void bootstrap_step(dfl_ctx* c, c64* f)
{
    const long F = c->field_elems;
    const int Ns = c->p.Ns;
    const double m = c->p.m0_setup, tol = c->p.little_tol_in;
    const dfl_prec lp = c->p.little_prec;
    // t_l = Phi A^-1 Phi^+ psi_l, and psi_l <- P_L psi_l = psi_l - D t_l
    for (int l = 0; l < Ns; ++l) {
        c64* fl = f + (long)l * F;
        c64* tl = c->bootT + (long)l * F;
        coarse(c, fl, tl, tol, lp);
        dirac64_sub(c, fl, tl, c->t1, m);
        launch_copy<double>(c->t1, fl, F, c->stream);
    }
    // chi = M_sap P_L psi for all fields at once
    {
        struct SetupSweeps {
            dfl_ctx* c;
            explicit SetupSweeps(dfl_ctx* cc) : c(cc) { c->sap_prof_cls = DFL_PROF_SETUP_SAP; }
            ~SetupSweeps() { c->sap_prof_cls = DFL_PROF_SAP; }
        } setup_sweeps(c);
        if (c->p.sap_prec == DFL_F64) {
            sap_apply(c, f, c->tN, m, Ns);
            launch_copy<double>(c->tN, f, F * Ns, c->stream);
        } else {
            sap_apply(c, f, f, m, Ns);  // FP32 path: staged through s32a/s32b
        }
    }
    // psi_l <- chi_l - Phi A^-1 Phi^+ D chi_l + t_l
    for (int l = 0; l < Ns; ++l) {
        c64* fl = f + (long)l * F;
        dirac64(c, fl, c->t1, m);
        coarse(c, c->t1, c->t2, tol, lp);
        launch_sub<double>(fl, c->t2, fl, F, c->stream);
        launch_add<double>(fl, c->bootT + (long)l * F, fl, F, c->stream);
    }
    launch_finite_check<double>(f, F * Ns, c->dflag, c->stream);
    launch_norm2_b<double>(f, F, Ns, F, c->red, c->dnorm, 2, nullptr, c->stream);
    launch_scale_invsqrt_b<double>(f, F, Ns, F, c->dnorm, 2, nullptr, c->stream);
}

}  // namespace
}  // namespace dfl

using namespace dfl;

#define API_BEGIN try {
#define API_END                                                                                                    \
    return DFL_OK;                                                                                                 \
    }                                                                                                              \
    catch (const dfl::Error& e)                                                                                    \
    {                                                                                                              \
        dfl::g_last_error = e.msg;                                                                                 \
        return e.code;                                                                                             \
    }                                                                                                              \
    catch (const std::bad_alloc&)                                                                                  \
    {                                                                                                              \
        dfl::g_last_error = "host allocation failed";                                                             \
        return DFL_ENOMEM;                                                                                         \
    }                                                                                                              \
    catch (...)                                                                                                    \
    {                                                                                                              \
        dfl::g_last_error = "unexpected internal error";                                                          \
        return DFL_EHIP;                                                                                           \
    }

extern "C" {

void dfl_default_params(dfl_params* p)
{
    if (!p)
        return;
    std::memset(p, 0, sizeof(*p));
    for (int mu = 0; mu < 4; ++mu) {
        p->sap_block[mu] = 4;
        p->dfl_block[mu] = 4;
    }
    p->Ns = 20;
    p->ncy = 5;
    p->nmr = 4;
    p->nkv = 16;
    p->n_inviter = 3;
    p->maxiter = 1000;
    p->nrhs_max = 1;
    p->little_nkv = 32;
    p->little_maxiter = 2000;
    p->solver = DFL_SOLVER_DFL_SAP_GCR;
    p->m0 = 0.0;
    p->m0_setup = 0.0;
    p->tol = 1e-10;
    p->little_tol_in = 1e-6;
    p->little_tol_out = 1e-12;
    p->link_prec = DFL_F64;
    p->sap_prec = DFL_F64;
    p->little_prec = DFL_F64;
    p->little_grid = 0;
    p->little_adapt = 1;
    p->little_eo = 1;
    p->little_gdefl = 1;
    p->csw = 0.0;
    p->antiperiodic = 0;
    p->n_boot = 0;
}

const char* dfl_last_error(void) { return dfl::g_last_error.c_str(); }

int dfl_profile_enable(dfl_ctx* c, int on)
{
    API_BEGIN
    need_ctx(c);
    prof_collect(c);
    c->prof_on = on != 0;
    API_END
}

int dfl_profile_read(dfl_ctx* c, double* seconds, long long* launches, long long* little_iters)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(seconds, "seconds");
    need_ptr(launches, "launches");
    prof_collect(c);
    for (int k = 0; k < DFL_PROF_NCLASS; ++k) {
        seconds[k] = c->prof_t[k];
        launches[k] = c->prof_n[k];
        c->prof_t[k] = 0.0;
        c->prof_n[k] = 0;
    }
    if (little_iters)
        *little_iters = c->prof_little_iters;
    c->prof_little_iters = 0;
    API_END
}

int dfl_residual_history(const dfl_ctx* c, double* out, int max)
{
    if (!c || max < 0 || (max > 0 && !out))
        return -1;
    int n = (int)c->history.size();
    for (int i = 0; i < n && i < max; ++i)
        out[i] = c->history[(size_t)i];
    return n;
}

int dfl_create(dfl_ctx** out, const dfl_params* p, void* hip_stream)
{
    dfl_ctx* c = nullptr;
    API_BEGIN
    need_ptr(out, "ctx");
    need_ptr(p, "params");
    *out = nullptr;
    validate(*p);
    c = new dfl_ctx();
    c->p = *p;
    c->stream = static_cast<hipStream_t>(hip_stream);
    HIPCHECK(hipGetDevice(&c->device));
    c->g = make_geom(p->dims, p->dfl_block);
    c->g.tsign = p->antiperiodic ? -1 : 1;
    c->V = c->g.V;
    c->field_elems = 12 * c->V;
    SapGeom& sg = c->sg;
    for (int mu = 0; mu < 4; ++mu) {
        sg.sb[mu] = p->sap_block[mu];
        sg.nsb[mu] = p->dims[mu] / p->sap_block[mu];
    }
    sg.lstr[3] = 1;
    for (int mu = 2; mu >= 0; --mu)
        sg.lstr[mu] = sg.lstr[mu + 1] * sg.sb[mu + 1];
    sg.Vsb = sg.sb[0] * sg.sb[1] * sg.sb[2] * sg.sb[3];
    sg.n_per_colour = sg.nsb[0] * sg.nsb[1] * sg.nsb[2] * sg.nsb[3] / 2;
    {
        // one-field sweeps: lane pairs (one block per CU) while a colour has
        // fewer than four blocks per CU, one lane per site (two blocks per CU)
        // beyond; measured on MI355X with 4^4 blocks: 128 and 256 blocks per
        // colour 11% faster with lane pairs, 4096 27% faster with one lane
        int cus = 0;
        HIPCHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
        sg.one_rl = sg.n_per_colour >= 4 * cus ? 1 : 0;
    }

    const long V = c->V, F = c->field_elems;
    const long N = (long)c->g.Nb * p->Ns;
    try {
        c->U64 = alloc_dev<c64>(c, (size_t)24 * V);
        c->U32 = alloc_dev<c32>(c, (size_t)24 * V);
        c->Ubf = alloc_dev<uint32_t>(c, (size_t)24 * V);
        if (p->csw != 0.0) {
            c->Cl64 = alloc_dev<c64>(c, (size_t)kCloverComp * V);
            c->Cl32 = alloc_dev<c32>(c, (size_t)kCloverComp * V);
        }
        c->Phi = alloc_dev<c64>(c, (size_t)p->Ns * F);
        if (p->little_prec == DFL_F32)
            c->Phi32 = alloc_dev<c32>(c, (size_t)p->Ns * F);
        c->A64 = alloc_dev<c64>(c, (size_t)c->g.Nb * 9 * p->Ns * p->Ns);
        c->A32 = alloc_dev<c32>(c, (size_t)c->g.Nb * 9 * p->Ns * p->Ns);
        c->At64 = alloc_dev<c64>(c, (size_t)c->g.Nb * 9 * p->Ns * p->Ns);
        c->At32 = alloc_dev<c32>(c, (size_t)c->g.Nb * 9 * p->Ns * p->Ns);
        if (p->little_eo) {
            c->Mt64 = alloc_dev<c64>(c, (size_t)c->g.Nb * 9 * p->Ns * p->Ns);
            c->Mt32 = alloc_dev<c32>(c, (size_t)c->g.Nb * 9 * p->Ns * p->Ns);
            c->lw1 = alloc_dev<c64>(c, (size_t)p->nrhs_max * N);  // one vector per source
            c->lw2 = alloc_dev<c64>(c, (size_t)p->nrhs_max * N);
            if (p->little_gdefl && p->Ns <= kMaxLittleDefl) {
                c->gsR = alloc_dev<c64>(c, (size_t)c->g.Nb * p->Ns * p->Ns);
                c->gU = alloc_dev<c64>(c, (size_t)p->Ns * N);
                c->gW = alloc_dev<c64>(c, (size_t)p->Ns * N);
                c->gQ = alloc_dev<c64>(c, (size_t)p->Ns * N);
                c->gZ = alloc_dev<c64>(c, (size_t)p->Ns * N);
                c->gQ32 = alloc_dev<c32>(c, (size_t)p->Ns * N);
                c->gZ32 = alloc_dev<c32>(c, (size_t)p->Ns * N);
                c->gC = alloc_dev<c64>(c, (size_t)p->Ns * p->Ns);
                c->gAinv = alloc_dev<double>(c, (size_t)2 * p->Ns * p->Ns);
                c->gGw = alloc_dev<double>(c, (size_t)2 * p->Ns * p->Ns);
            }
        }
        const long R = p->nrhs_max;
        c->xi = alloc_dev<c64>(c, (size_t)p->nkv * R * F);
        c->chi = alloc_dev<c64>(c, (size_t)p->nkv * R * F);
        c->rho = alloc_dev<c64>(c, R * F);
        c->acc = alloc_dev<c64>(c, R * F);
        c->t1 = alloc_dev<c64>(c, R * F);
        c->t2 = alloc_dev<c64>(c, R * F);
        c->t3 = alloc_dev<c64>(c, R * F);
        const long nf = p->nrhs_max > p->Ns ? p->nrhs_max : p->Ns;  // multi-field Schwarz buffers
        c->s32a = alloc_dev<c32>(c, (size_t)nf * F);
        c->s32b = alloc_dev<c32>(c, (size_t)nf * F);
        c->s32c = alloc_dev<c32>(c, F);
        if (p->sap_prec == DFL_F64)
            c->tN = alloc_dev<c64>(c, (size_t)p->Ns * F);
        if (p->n_boot > 0) {
            c->bootF = alloc_dev<c64>(c, (size_t)p->Ns * F);
            c->bootT = alloc_dev<c64>(c, (size_t)p->Ns * F);
        }
        c->lxi = alloc_dev<c64>(c, (size_t)p->little_nkv * R * N);
        c->lchi = alloc_dev<c64>(c, (size_t)p->little_nkv * R * N);
        c->lr = alloc_dev<c64>(c, R * N);
        c->lx = alloc_dev<c64>(c, R * N);
        c->lw = alloc_dev<c64>(c, R * N);
        c->lt = alloc_dev<c64>(c, N);
        c->lw32 = alloc_dev<c32>(c, R * N);
        c->lx32 = alloc_dev<c32>(c, R * N);
        c->lgrid = little_gcr_grid(c->g, p->little_grid);
        c->lgrid_multi = little_gcr_multi_grid(c->g, p->little_grid);
        // every workgroup of the grid-barrier kernels must be resident at
        // once (graph replays launch them as ordinary kernels)
        c->lgrid = std::min(c->lgrid, little_gcr_resident_limit(false));
        c->lgrid_multi = std::min(c->lgrid_multi, little_gcr_resident_limit(true));
        if (c->lgrid < 1 || c->lgrid_multi < 1)
            fail(DFL_EHIP, "the little GCR kernels cannot be resident on this device");
        size_t part = little_gcr_partial_doubles(c->lgrid);
        if (R > 1) {
            size_t nfin = 0, nac = 0;
            part = std::max(part, little_gcr_multi_doubles(c->lgrid_multi, (int)R, &nfin, &nac));
            c->lfin = alloc_dev<double>(c, nfin);
            c->lacoef = alloc_dev<double>(c, nac);
        }
        c->lpart = alloc_dev<double>(c, part);
        c->lstats = alloc_dev<int>(c, 4);
        c->lbar_count = alloc_dev<unsigned>(c, 64);
        c->lbar_gen = alloc_dev<unsigned long long>(c, 32);
        const long RM = std::max<long>(R, max_multi_fields(c));  // fields normalised in one launch
        c->red = alloc_dev<double>(c, (size_t)kMaxDot * kRedBlocks * 2 * RM);
        c->dnorm = alloc_dev<double>(c, (size_t)2 * RM);
        c->dscal = alloc_dev<double>(c, S_TOTAL * R);
        c->dflag = alloc_dev<int>(c, 4);
        c->dact = alloc_dev<int>(c, kMaxLittleRhs);
        c->dact2 = alloc_dev<int>(c, kMaxLittleRhs);
        c->dtol = alloc_dev<double>(c, 2);
        HIPCHECK(hipHostMalloc((void**)&c->htol, sizeof(double) * 2, hipHostMallocDefault));
        HIPCHECK(hipHostMalloc((void**)&c->hscal, sizeof(double) * S_TOTAL * R, hipHostMallocDefault));
        HIPCHECK(hipHostMalloc((void**)&c->hact, sizeof(int) * kMaxLittleRhs, hipHostMallocDefault));
        HIPCHECK(hipMemsetAsync(c->dscal, 0, sizeof(double) * S_TOTAL * R, c->stream));
        HIPCHECK(hipMemsetAsync(c->dact, 0, sizeof(int) * kMaxLittleRhs, c->stream));
        HIPCHECK(hipMemsetAsync(c->dflag, 0, sizeof(int) * 4, c->stream));
        HIPCHECK(hipMemsetAsync(c->lstats, 0, sizeof(int) * 4, c->stream));
        HIPCHECK(hipMemsetAsync(c->lbar_count, 0, sizeof(unsigned) * 64, c->stream));
        HIPCHECK(hipMemsetAsync(c->lbar_gen, 0, sizeof(unsigned long long) * 32, c->stream));
        sync(c);
    } catch (...) {
        free_all(c);
        delete c;
        throw;
    }
    *out = c;
    API_END
}

int dfl_destroy(dfl_ctx* c)
{
    API_BEGIN
    if (!c)
        return DFL_OK;
    (void)hipStreamSynchronize(c->stream);
    if (c->gstream)
        (void)hipStreamSynchronize(c->gstream);
    drop_graphs(c);
    for (hipEvent_t e : c->gev)
        if (e)
            (void)hipEventDestroy(e);
    if (c->gstream)
        (void)hipStreamDestroy(c->gstream);
    for (auto& p : c->ev_pending) {
        (void)hipEventDestroy(p.second.first);
        (void)hipEventDestroy(p.second.second);
    }
    for (hipEvent_t e : c->ev_pool)
        (void)hipEventDestroy(e);
    free_all(c);
    delete c;
    API_END
}

long long dfl_field_bytes(const dfl_ctx* c, dfl_prec prec)
{
    if (!c)
        return -1;
    return (long long)c->field_elems * (prec == DFL_F64 ? 16 : 8);
}

int dfl_use_graphs(dfl_ctx* c, int on)
{
    API_BEGIN
    need_ctx(c);
    sync(c);
    if (!on)
        drop_graphs(c);
    if (on && !c->gstream) {
        HIPCHECK(hipStreamCreate(&c->gstream));
        HIPCHECK(hipEventCreateWithFlags(&c->gev[0], hipEventDisableTiming));
        HIPCHECK(hipEventCreateWithFlags(&c->gev[1], hipEventDisableTiming));
    }
    c->use_graph = on != 0;
    API_END
}

long long dfl_graph_replays(const dfl_ctx* c) { return c ? c->graph_replays : -1; }

int dfl_num_blocks(const dfl_ctx* c) { return c ? c->g.Nb : -1; }

int dfl_set_mass(dfl_ctx* c, double m0)
{
    API_BEGIN
    need_ctx(c);
    if (!std::isfinite(m0))
        fail(DFL_EINVAL, "mass must be finite");
    if (m0 != c->p.m0)
        drop_graphs(c);  // the mass is a kernel argument of the captured steps
    c->p.m0 = m0;
    if (c->have_subspace && m0 != c->m0_A) {
        // the basis is orthonormal, so A(m0') = A(m0) + (m0' - m0) 1
        launch_little_shift(c->g, c->A64, c->p.Ns, m0 - c->m0_A, c->stream);
        launch_little_copies(c->A64, c->A32, c->At64, c->At32, (long)c->g.Nb * 9, c->p.Ns, c->stream);
        c->m0_A = m0;
        prepare_eo(c);
        prepare_gdefl(c);
    }
    API_END
}

int dfl_set_gauge(dfl_ctx* c, const double* U)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(U, "U");
    sync(c);
    drop_graphs(c);  // captured steps hold the subspace state they were recorded with
    c->have_gauge = false;
    c->have_subspace = false;
    HIPCHECK(hipMemsetAsync(c->dflag, 0, sizeof(int), c->stream));
    launch_pack_gauge(c->g, reinterpret_cast<const c64*>(U), c->U64, c->U32, c->Ubf, c->dflag, c->stream);
    HIPCHECK(hipGetLastError());
    int flag = 0;
    HIPCHECK(hipMemcpyAsync(&flag, c->dflag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    sync(c);
    if (flag)
        fail(DFL_EINVAL, "gauge field: every link must be SU(3) (third row = conj(row0 x row1) to 1e-12)");
    if (c->Cl64) {
        launch_clover_field(c->g, links64(c), c->p.csw, c->Cl64, c->Cl32, c->stream);
        HIPCHECK(hipGetLastError());
    }
    c->have_gauge = true;
    API_END
}

int dfl_pack(dfl_ctx* c, const double* canon, void* nat, int nrhs, dfl_prec prec)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(canon, "canon");
    need_ptr(nat, "native");
    if (nrhs < 1)
        fail(DFL_EINVAL, "nrhs must be >= 1");
    if (prec == DFL_F64)
        launch_pack_field64(c->g, reinterpret_cast<const c64*>(canon), static_cast<c64*>(nat), nrhs, c->stream);
    else if (prec == DFL_F32)
        launch_pack_field32(c->g, reinterpret_cast<const c64*>(canon), static_cast<c32*>(nat), nrhs, c->stream);
    else
        fail(DFL_EINVAL, "fields are F64 or F32");
    HIPCHECK(hipGetLastError());
    API_END
}

int dfl_unpack(dfl_ctx* c, const void* nat, double* canon, int nrhs, dfl_prec prec)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(canon, "canon");
    need_ptr(nat, "native");
    if (nrhs < 1)
        fail(DFL_EINVAL, "nrhs must be >= 1");
    if (prec == DFL_F64)
        launch_unpack_field64(c->g, static_cast<const c64*>(nat), reinterpret_cast<c64*>(canon), nrhs, c->stream);
    else if (prec == DFL_F32)
        launch_unpack_field32(c->g, static_cast<const c32*>(nat), reinterpret_cast<c64*>(canon), nrhs, c->stream);
    else
        fail(DFL_EINVAL, "fields are F64 or F32");
    HIPCHECK(hipGetLastError());
    API_END
}

int dirac_apply(dfl_ctx* c, const void* psi, void* out, int nrhs, dfl_prec prec)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(psi, "psi");
    need_ptr(out, "out");
    need_gauge(c);
    need_nrhs(c, nrhs);
    if (psi == out)
        fail(DFL_EINVAL, "psi and out must not overlap");
    ProfScope ps(c, DFL_PROF_DIRAC);
    if (prec == DFL_F64)
        launch_dirac64(c->g, links64(c), static_cast<const c64*>(psi), static_cast<c64*>(out), nrhs, c->p.m0, 0, 0,
                       0, c->stream, c->Cl64);
    else if (prec == DFL_F32 && c->p.link_prec == DFL_BF16)
        launch_dirac_bf16(c->g, linksbf(c), static_cast<const c32*>(psi), static_cast<c32*>(out), nrhs,
                          (float)c->p.m0, c->stream, c->Cl32);
    else if (prec == DFL_F32)
        launch_dirac32(c->g, links32(c), static_cast<const c32*>(psi), static_cast<c32*>(out), nrhs, (float)c->p.m0,
                       c->stream, c->Cl32);
    else
        fail(DFL_EINVAL, "dirac_apply precision must be F64 or F32");
    HIPCHECK(hipGetLastError());
    API_END
}

int sap_precond(dfl_ctx* c, const void* rho, void* psi, int nrhs)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(rho, "rho");
    need_ptr(psi, "psi");
    need_gauge(c);
    need_nrhs(c, nrhs);
    if (rho == psi)
        fail(DFL_EINVAL, "rho and psi must not overlap");
    sap_apply(c, static_cast<const c64*>(rho), static_cast<c64*>(psi), c->p.m0, nrhs);
    HIPCHECK(hipGetLastError());
    API_END
}

int dfl_setup(dfl_ctx* c, const void* init, int n_init)
{
    API_BEGIN
    const auto ts0 = std::chrono::steady_clock::now();
    need_ctx(c);
    need_ptr(init, "init fields (the caller draws the random start fields)");
    need_gauge(c);
    if (n_init != c->p.Ns)
        fail(DFL_EINVAL, "n_init must equal Ns");
    const int Ns = c->p.Ns;
    const int nb = c->p.n_boot;
    // captured GCR steps keep the even-odd and global-deflation state (and
    // the buffers of Q and Z) of the subspace they were recorded with
    sync(c);
    drop_graphs(c);
    c->have_subspace = false;
    // the fields are relaxed in Phi itself, or (bootstrapped iteration) kept
    // apart from the intermediate subspaces built from them
    c64* fields = nb > 0 ? c->bootF : c->Phi;
    HIPCHECK(hipMemsetAsync(c->dflag, 0, sizeof(int) * 4, c->stream));
    // inverse iteration, eq. (5.1): psi_l <- M_sap psi_l, normalised; the
    // Schwarz sweeps relax all Ns fields in one launch each. The first step
    // reads the caller's fields; the last normalisation is left out, since
    // everything built from the fields (their block Gram-Schmidt, the
    // global deflation modes, a bootstrapped step) depends only on each
    // field's direction.
    inverse_iterate(c, static_cast<const c64*>(init), fields, Ns, c->p.n_inviter - nb, false);
    // bootstrapped steps (section 5.3): the current fields deflate the
    // approximate solve of the next step
    for (int b = 0; b < nb; ++b) {
        build_subspace(c, fields, c->p.m0_setup);
        bootstrap_step(c, fields);
    }
    build_subspace(c, fields, c->p.m0);  // synchronises
    c->have_subspace = true;
    c->t_setup_last = std::chrono::duration<double>(std::chrono::steady_clock::now() - ts0).count();
    API_END
}

int dfl_get_basis(dfl_ctx* c, void* phi)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(phi, "phi");
    need_subspace(c);
    HIPCHECK(hipMemcpyAsync(phi, c->Phi, sizeof(c64) * c->field_elems * c->p.Ns, hipMemcpyDeviceToDevice,
                            c->stream));
    API_END
}

int dfl_get_little(dfl_ctx* c, double* A)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(A, "A");
    need_subspace(c);
    HIPCHECK(hipMemcpyAsync(A, c->A64, sizeof(c64) * c->g.Nb * 9 * c->p.Ns * c->p.Ns, hipMemcpyDeviceToDevice,
                            c->stream));
    API_END
}

int little_dirac_apply(dfl_ctx* c, const void* v, void* w, int nrhs, dfl_prec prec)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(v, "v");
    need_ptr(w, "w");
    need_subspace(c);
    need_nrhs(c, nrhs);
    if (v == w)
        fail(DFL_EINVAL, "v and w must not overlap");
    if (prec == DFL_F64)
        launch_little_apply<double>(c->g, c->A64, c->p.Ns, static_cast<const c64*>(v), static_cast<c64*>(w), nrhs,
                                    c->stream);
    else if (prec == DFL_F32 && nrhs == 1)
        launch_little_apply<float>(c->g, c->A32, c->p.Ns, static_cast<const c32*>(v), static_cast<c32*>(w), 1,
                                   c->stream);
    else if (prec == DFL_F32)
        launch_little_apply_mfma(c->g, c->At32, c->p.Ns, static_cast<const c32*>(v), static_cast<c32*>(w), nrhs,
                                 c->stream);
    else
        fail(DFL_EINVAL, "little vectors are F64 or F32");
    HIPCHECK(hipGetLastError());
    API_END
}

int little_solve(dfl_ctx* c, const void* w, void* v, double tol, int* iters)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(w, "w");
    need_ptr(v, "v");
    need_subspace(c);
    if (!(tol > 0.0))
        fail(DFL_EINVAL, "tol must be positive");
    if (w == v)
        fail(DFL_EINVAL, "w and v must not overlap");
    reset_little_stats(c);
    little_solve_impl(c, static_cast<const c64*>(w), static_cast<c64*>(v), tol, DFL_F64);
    int st[3];
    read_little_stats(c, st);
    if (iters)
        *iters = st[0];
    if (st[2]) {
        g_last_error = "little solve did not converge within little_maxiter";
        return DFL_NOT_CONVERGED;
    }
    API_END
}

int deflate_project(dfl_ctx* c, dfl_proj which, const void* in, void* out, int nrhs)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(in, "in");
    need_ptr(out, "out");
    need_subspace(c);
    need_nrhs(c, nrhs);
    if (in == out)
        fail(DFL_EINVAL, "in and out must not overlap");
    const long F = c->field_elems;
    const double tol = c->p.little_tol_out;
    const c64* x = static_cast<const c64*>(in);
    c64* y = static_cast<c64*>(out);
    switch (which) {
    case DFL_PROJ_PL:
        apply_PL(c, x, y, tol, DFL_F64, c->t1, c->t2, nrhs);
        break;
    case DFL_PROJ_PR:
        dirac64(c, x, c->t1, c->p.m0, nrhs);
        coarse(c, c->t1, c->t2, tol, DFL_F64, nrhs);
        launch_sub<double>(x, c->t2, y, F * nrhs, c->stream);
        break;
    case DFL_PROJ_P:
        launch_restrict64(c->g, c->Phi, c->p.Ns, x, static_cast<c64*>(c->lw), nrhs, c->stream);
        launch_prolong64(c->g, c->Phi, c->p.Ns, static_cast<c64*>(c->lw), y, nrhs, c->stream);
        break;
    case DFL_PROJ_COARSE:
        coarse(c, x, y, tol, DFL_F64, nrhs);
        break;
    default:
        fail(DFL_EINVAL, "unknown projector");
    }
    HIPCHECK(hipGetLastError());
    API_END
}

int solve(dfl_ctx* c, const void* eta_v, void* psi_v, int nrhs, dfl_info* info)
{
    int worst = DFL_OK;
    API_BEGIN
    need_ctx(c);
    need_ptr(eta_v, "eta");
    need_ptr(psi_v, "psi");
    need_gauge(c);
    need_nrhs(c, nrhs);
    if (eta_v == psi_v)
        fail(DFL_EINVAL, "eta and psi must not overlap");
    const bool deflate = c->p.solver == DFL_SOLVER_DFL_SAP_GCR;
    const bool use_sap = c->p.solver != DFL_SOLVER_GCR;
    if (deflate)
        need_subspace(c);
    const long F = c->field_elems;
    const double m0 = c->p.m0;
    const int nb = nrhs;
    auto t0 = std::chrono::steady_clock::now();
    // per-class kernel seconds of this solve (event timers, profiling on)
    double prof0[DFL_PROF_NCLASS] = {0};
    if (c->prof_on) {
        prof_collect(c);
        for (int k = 0; k < DFL_PROF_NCLASS; ++k)
            prof0[k] = c->prof_t[k];
    }
    const c64* eta = static_cast<const c64*>(eta_v);
    c64* psi = static_cast<c64*>(psi_v);
    HIPCHECK(hipMemsetAsync(c->dflag, 0, sizeof(int), c->stream));
    launch_finite_check<double>(eta, F * nb, c->dflag, c->stream);
    int flag = 0;
    HIPCHECK(hipMemcpyAsync(&flag, c->dflag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    std::vector<double> eta_n = host_norm2_b(c, eta, F, nb);
    for (auto& q : eta_n)
        q = std::sqrt(q);
    if (flag)
        fail(DFL_ENONFINITE, "non-finite entries in the source");
    reset_little_stats(c);
    // initial residues: P_L eta (deflated) or eta
    if (deflate)
        apply_PL(c, eta, c->rho, c->p.little_tol_out, DFL_F64, c->t1, c->t2, nb);
    else
        launch_copy<double>(eta, c->rho, F * nb, c->stream);
    GcrVecs v{c->xi, c->chi, c->rho, c->acc};
    const dfl_prec lp = c->p.little_prec;
    auto precond = [&](const c64* r, c64* x, int n_b) {
        if (use_sap)
            sap_apply(c, r, x, m0, n_b);
        else
            launch_copy<double>(r, x, F * n_b, c->stream);
    };
    const bool adapt = deflate && c->p.little_adapt;
    auto op = [&](const c64* x, c64* y, int n_b) {
        if (deflate) {
            dirac64(c, x, c->t3, m0, n_b);
            apply_PL(c, c->t3, y, c->p.little_tol_in, lp, c->t1, c->t2, n_b, adapt ? c->dtol : nullptr);
        } else {
            dirac64(c, x, y, m0, n_b);
        }
    };
    auto recompute = [&](const c64* x, c64* r, int n_b) {
        if (deflate) {
            dirac64_sub(c, eta, x, c->t3, m0, n_b);
            apply_PL(c, c->t3, r, c->p.little_tol_out, DFL_F64, c->t1, c->t2, n_b);
        } else {
            dirac64_sub(c, eta, x, r, m0, n_b);
        }
    };
    // With inexact projections inside the cycle (little solves to
    // little_tol_in), the recursively updated residue stops tracking the
    // true one once it has fallen by about that factor; the cycle is then
    // ended early and the residue recomputed (appendix A.5).
    const double cycle_floor = deflate ? 10.0 * c->p.little_tol_in : 0.0;
    c->history.clear();
    // Adapted precision inside a cycle (appendix A.5): the residue, hence the
    // field the projector acts on, has fallen by `ratio` since the cycle
    // began, so a relative little-solve tolerance little_tol_in / ratio keeps
    // the absolute error of the projection fixed (capped at 1e-2).
    auto inner_tol = [&](double ratio) { return std::min(1e-2, c->p.little_tol_in / std::max(ratio, 1e-300)); };
    std::vector<GcrResult> res = gcr_run(c, F, nb, c->p.nkv, c->p.maxiter, c->p.tol, eta_n, v, precond, op,
                                         recompute, cycle_floor, &c->history,
                                         adapt ? std::function<double(double)>(inner_tol) : nullptr);
    // final solutions: psi = acc + Phi A^-1 Phi^+ (eta - D acc)   (eq. (3.10) with P_R)
    if (deflate) {
        dirac64_sub(c, eta, c->acc, c->t3, m0, nb);
        coarse(c, c->t3, c->t1, c->p.little_tol_out, DFL_F64, nb);
        launch_add<double>(c->acc, c->t1, psi, F * nb, c->stream);
    } else {
        launch_copy<double>(c->acc, psi, F * nb, c->stream);
    }
    // true residuals in FP64
    dirac64_sub(c, eta, psi, c->t2, m0, nb);
    std::vector<double> rr = host_norm2_b(c, c->t2, F, nb);
    auto t1 = std::chrono::steady_clock::now();
    if (c->prof_on)
        prof_collect(c);
    int ls[3] = {0, 0, 0};
    read_little_stats(c, ls);
    for (int b = 0; b < nb; ++b) {
        int status = res[b].status;
        double rel = eta_n[b] > 0.0 ? std::sqrt(rr[b]) / eta_n[b] : 0.0;
        if (status == DFL_OK && rel > c->p.tol)
            status = DFL_NOT_CONVERGED;
        if (status != DFL_OK)
            worst = status;
        if (info) {
            dfl_info& q = info[b];
            q.status = status;
            q.n_gcr = res[b].iters;
            q.n_restarts = res[b].restarts;
            q.n_little = ls[0];
            q.n_little_solves = ls[1];
            q.rel_residual = rel;
            q.t_solve = std::chrono::duration<double>(t1 - t0).count();
            q.t_setup = c->t_setup_last;
            q.t_sap = q.t_dirac = q.t_proj = q.t_little = -1.0;
            if (c->prof_on) {
                q.t_sap = c->prof_t[DFL_PROF_SAP] - prof0[DFL_PROF_SAP];
                q.t_dirac = c->prof_t[DFL_PROF_DIRAC] - prof0[DFL_PROF_DIRAC];
                q.t_proj = c->prof_t[DFL_PROF_PROJECT] - prof0[DFL_PROF_PROJECT];
                q.t_little = c->prof_t[DFL_PROF_LITTLE] - prof0[DFL_PROF_LITTLE];
            }
        }
    }
    if (worst != DFL_OK) {
        g_last_error = "solve: tolerance not reached within maxiter";
        return worst;
    }
    API_END
}

// ------------------------------------------------------ start-field network

int dfl_inverse_iteration(dfl_ctx* c, void* fields, int n, int steps)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(fields, "fields");
    need_gauge(c);
    if (n < 1 || n > max_multi_fields(c))
        fail(DFL_EINVAL, "n must be in 1..Ns (FP64 Schwarz) or 1..max(Ns, nrhs_max)");
    if (steps < 0)
        fail(DFL_EINVAL, "steps must be >= 0");
    HIPCHECK(hipMemsetAsync(c->dflag, 0, sizeof(int) * 4, c->stream));
    inverse_iterate(c, static_cast<c64*>(fields), static_cast<c64*>(fields), n, steps);
    int flag[4];
    HIPCHECK(hipMemcpyAsync(flag, c->dflag, sizeof(flag), hipMemcpyDeviceToHost, c->stream));
    sync(c);
    if (flag[0] & 1)
        fail(DFL_ENONFINITE, "non-finite entries in the fields");
    API_END
}

int net_features(dfl_ctx* c, const float* noise, float* x)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(noise, "noise");
    need_ptr(x, "x");
    need_gauge(c);
    launch_net_features(c->g, c->U64, noise, x, c->stream);
    HIPCHECK(hipGetLastError());
    API_END
}

int conv4d_forward(dfl_ctx* c, const float* in, int cin, const float* W, const float* b, int cout, float* z, float* a)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(in, "in");
    need_ptr(W, "W");
    need_ptr(z, "z");
    if (cin < 1 || cin > kNetMaxCin || cout < 1 || cout > kNetMaxCout)
        fail(DFL_EINVAL, "channels: 1 <= cin <= 96, 1 <= cout <= 576");
    if (z == in || a == in)
        fail(DFL_EINVAL, "outputs must not overlap the input");
    launch_conv_forward(c->g, in, cin, W, b, cout, z, a, c->stream);
    HIPCHECK(hipGetLastError());
    API_END
}

int conv4d_forward_bf16(dfl_ctx* c, const float* in, int cin, const float* W, const float* b, int cout, float* z,
                        float* a)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(in, "in");
    need_ptr(W, "W");
    need_ptr(z, "z");
    if (cin < 1 || cin > kNetMaxCin || cout < 1 || cout > kNetMaxCout)
        fail(DFL_EINVAL, "channels: 1 <= cin <= 96, 1 <= cout <= 576");
    if (z == in || a == in)
        fail(DFL_EINVAL, "outputs must not overlap the input");
    if (!conv_bf16_fits(c->g))
        fail(DFL_EINVAL, "the BF16 convolution needs L3 % 32 == 0 and L2 % 4 == 0");
    c->net_wbf = grow<uint16_t>(c, c->net_wbf, c->net_wbf_n, conv_bf16_weight_elems(cin, cout));
    launch_conv_forward_bf16(c->g, in, cin, W, b, cout, z, a, c->net_wbf, c->stream);
    HIPCHECK(hipGetLastError());
    API_END
}

int conv4d_backward(dfl_ctx* c, const float* in, int cin, const float* W, int cout, const float* g, float* dW,
                    float* db, float* din, const float* z_in)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(in, "in");
    need_ptr(W, "W");
    need_ptr(g, "g");
    need_ptr(dW, "dW");
    need_ptr(db, "db");
    if (cin < 1 || cin > kNetMaxCin || cout < 1 || cout > kNetMaxCout)
        fail(DFL_EINVAL, "channels: 1 <= cin <= 96, 1 <= cout <= 576");
    if (din && (din == g || din == in))
        fail(DFL_EINVAL, "din must not overlap g or in");
    long chunk = 0;
    int nchunk = 0;
    const size_t need = conv_wgrad_chunk_floats(c->g, cin, cout, &chunk, &nchunk);
    c->net_part = grow<float>(c, c->net_part, c->net_part_n, need);
    launch_conv_backward(c->g, in, cin, W, cout, g, dW, db, din, z_in, c->net_part, chunk, nchunk, c->stream);
    HIPCHECK(hipGetLastError());
    API_END
}

int conv4d_backward_noalloc(dfl_ctx* c, const float* in, int cin, const float* W, int cout, const float* g,
                            float* dW, float* db, float* din, const float* z_in)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(in, "in");
    need_ptr(W, "W");
    need_ptr(g, "g");
    need_ptr(dW, "dW");
    need_ptr(db, "db");
    if (cin < 1 || cin > kNetMaxCin || cout < 1 || cout > kNetMaxCout)
        fail(DFL_EINVAL, "channels: 1 <= cin <= 96, 1 <= cout <= 576");
    if (din && (din == g || din == in))
        fail(DFL_EINVAL, "din must not overlap g or in");
    long chunk = 0;
    int nchunk = 0;
    if (!conv_wgrad_chunk_fit(c->g, cin, cout, kNoAllocFloats, &chunk, &nchunk))
        fail(DFL_EINVAL, "conv4d_backward_noalloc: one chunk of the weight-gradient partial sums (81 cin cout "
                         "floats) exceeds the 64 MiB scratch");
    float* part = noalloc_scratch();
    launch_conv_backward(c->g, in, cin, W, cout, g, dW, db, din, z_in, part, chunk, nchunk, c->stream);
    HIPCHECK(hipGetLastError());
    API_END
}

int net_outputs_to_fields(dfl_ctx* c, const float* out, int Ns, void* fields)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(out, "out");
    need_ptr(fields, "fields");
    if (Ns < 1 || 24 * Ns > kNetMaxCout)
        fail(DFL_EINVAL, "Ns must be in 1..24");
    launch_out_to_fields(c->g, out, Ns, static_cast<c64*>(fields), c->stream);
    HIPCHECK(hipGetLastError());
    API_END
}

int net_fields_grad_to_outputs(dfl_ctx* c, const void* grad, int Ns, float* dout)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(grad, "grad");
    need_ptr(dout, "dout");
    if (Ns < 1 || 24 * Ns > kNetMaxCout)
        fail(DFL_EINVAL, "Ns must be in 1..24");
    launch_fields_to_out(c->g, static_cast<const c64*>(grad), Ns, dout, c->stream);
    HIPCHECK(hipGetLastError());
    API_END
}

int deficit_loss(dfl_ctx* c, const void* fields, int Ns, const void* targets, int K, double* loss, void* grad)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(fields, "fields");
    need_ptr(targets, "targets");
    need_ptr(loss, "loss");
    if (Ns < 1 || Ns > kLossMaxN || K < 1 || K > kLossMaxN)
        fail(DFL_EINVAL, "Ns and K must be in 1..32");
    if (Ns > 12 * c->g.Vb)
        fail(DFL_EINVAL, "Ns exceeds the dimension of a block");
    const long Nb = c->g.Nb;
    const size_t nY = (size_t)Nb * Ns * K;
    if (nY > c->loss_n || !c->loss_buf) {
        sync(c);
        if (c->loss_Y)
            HIPCHECK(hipFree(c->loss_Y));
        if (c->loss_buf)
            HIPCHECK(hipFree(c->loss_buf));
        if (c->loss_host)
            HIPCHECK(hipHostFree(c->loss_host));
        c->loss_Y = nullptr;
        c->loss_buf = nullptr;
        c->loss_host = nullptr;
        c->loss_n = 0;
        const size_t cap_Y = (size_t)Nb * kLossMaxN * kLossMaxN;
        const size_t cap_b = (size_t)Nb * kLossMaxN * 2 + kLossMaxN;
        c->loss_Y = alloc_dev<c64>(c, cap_Y);
        c->loss_buf = alloc_dev<double>(c, cap_b);
        HIPCHECK(hipHostMalloc((void**)&c->loss_host, sizeof(double) * cap_b, hipHostMallocDefault));
        c->loss_n = cap_Y;
    }
    double* tb2 = c->loss_buf;
    double* proj = tb2 + Nb * K;
    double* wk = proj + Nb * K;
    HIPCHECK(hipMemsetAsync(c->dflag, 0, sizeof(int) * 4, c->stream));
    launch_deficit_block(c->g, static_cast<const c64*>(fields), Ns, static_cast<const c64*>(targets), K, c->loss_Y,
                         tb2, proj, c->dflag, c->stream);
    HIPCHECK(hipGetLastError());
    int flag[4];
    HIPCHECK(hipMemcpyAsync(c->loss_host, tb2, sizeof(double) * Nb * K * 2, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(hipMemcpyAsync(flag, c->dflag, sizeof(flag), hipMemcpyDeviceToHost, c->stream));
    sync(c);
    if (flag[0] & 1)
        fail(DFL_ESINGULAR, "deficit loss: the fields are linearly dependent on a block");
    const double* h_tb2 = c->loss_host;
    const double* h_proj = h_tb2 + Nb * K;
    double* h_wk = c->loss_host + Nb * K * 2;
    double total = 0.0;
    for (int k = 0; k < K; ++k) {
        double tn2 = 0.0, pr = 0.0;
        for (long b = 0; b < Nb; ++b) {
            tn2 += h_tb2[b * K + k];
            pr += h_proj[b * K + k];
        }
        if (!(tn2 > 0.0))
            fail(DFL_EINVAL, "deficit loss: a target field is zero");
        total += (tn2 - pr) / tn2;
        h_wk[k] = 1.0 / (K * tn2);
    }
    *loss = total / K;
    if (grad) {
        HIPCHECK(hipMemcpyAsync(wk, h_wk, sizeof(double) * K, hipMemcpyHostToDevice, c->stream));
        launch_deficit_grad(c->g, static_cast<const c64*>(fields), Ns, static_cast<const c64*>(targets), K,
                            c->loss_Y, wk, static_cast<c64*>(grad), c->stream);
        HIPCHECK(hipGetLastError());
        sync(c);  // the weights live in the pinned mirror until the copy has run
    }
    API_END
}

int adam_update(dfl_ctx* c, float* theta, const float* g, float* m, float* v, long long n, int t, double lr, double b1,
                double b2, double eps)
{
    API_BEGIN
    need_ctx(c);
    need_ptr(theta, "theta");
    need_ptr(g, "g");
    need_ptr(m, "m");
    need_ptr(v, "v");
    if (t < 1 || n < 0 || !(lr > 0.0) || !(b1 >= 0.0 && b1 < 1.0) || !(b2 >= 0.0 && b2 < 1.0) || !(eps > 0.0))
        fail(DFL_EINVAL, "adam: t >= 1, n >= 0, lr > 0, 0 <= b1, b2 < 1, eps > 0");
    const double c1 = 1.0 - std::pow(b1, t), c2 = 1.0 - std::pow(b2, t);
    launch_adam(theta, g, m, v, (long)n, (float)lr, (float)b1, (float)b2, (float)eps, (float)c1, (float)c2,
                c->stream);
    HIPCHECK(hipGetLastError());
    API_END
}

}  // extern "C"
