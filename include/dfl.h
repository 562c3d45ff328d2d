/*
 * dfl.h -- C ABI of the MI355X (gfx950) deflated, Schwarz-preconditioned GCR
 * solver for the lattice Wilson-Dirac equation D psi = eta.
 *
 * The method is that of M. Luescher, "Local coherence and deflation of the
 * low quark modes in lattice QCD": flexible GCR (section 6.2) on the
 * right-preconditioned deflated equation P_L D M_sap phi = P_L eta
 * (eq. (6.2)), with a block-projected deflation subspace (sections 4.1-4.2)
 * built by inverse iteration (eq. (5.1)) and the little Dirac operator of
 * eqs. (3.2)/(A.1).
 *
 * Operator. D is the O(a)-improved Wilson operator of section 2.1:
 *   (D psi)(x) = (4 + m0) psi(x) + csw (i/4) sum_{mu,nu} sigma_{mu nu} Fhat_{mu nu}(x) psi(x)
 *                - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu) ]
 * with the chiral basis g_mu = [[0, e_mu], [e_mu^+, 0]], e_0 = -1,
 * e_k = -i sigma_k (so g_5 = diag(1, 1, -1, -1)), sigma_{mu nu} = (i/2)[g_mu, g_nu],
 * Fhat_{mu nu}(x) = (Q_{mu nu}(x) - Q_{mu nu}(x)^+)/8 with Q_{mu nu} the sum of the
 * four plaquettes in the (mu, nu) plane around x. csw = 0 (the default) is
 * the plain Wilson operator. Space is periodic; time (direction 0) periodic
 * or antiperiodic (dfl_params.antiperiodic).
 *
 * Canonical layouts (host-side convention, also accepted on the device):
 *   site s = ((x0*L1 + x1)*L2 + x2)*L3 + x3 (x0 slowest), V sites;
 *   quark field: complex128 [V][12], component 3*spin + colour;
 *   gauge field: complex128 [V][4][3][3], U[s][mu][row][col], link x -> x+mu.
 * Native layouts (what the compute calls take) are produced by dfl_pack and
 * undone by dfl_unpack; they are structure-of-arrays, blocked by the
 * deflation block, and opaque to the caller except for their size:
 *   native quark field = dfl_field_bytes(ctx, prec) bytes per right-hand side,
 *   nrhs fields back to back.
 *   native little vector = Nb*Ns complex (FP64: 16 B, FP32: 8 B each) per
 *   right-hand side, entry [block][k] (k fastest), blocks lexicographic in the
 *   block coordinates (x0 slowest), nrhs vectors back to back.
 *
 * Memory and streams. Every pointer argument named *_dev is DEVICE memory on
 * the context's device; the caller owns it and keeps it alive for the call.
 * The context owns every internal buffer (allocated in dfl_create and
 * dfl_setup). All work is ordered on the stream given to dfl_create; calls
 * return after enqueueing unless stated otherwise (solve and dfl_setup
 * synchronise). A context must not be used from two threads at once.
 *
 * Errors. Every call returns a dfl_status. Negative: nothing valid was
 * written; DFL_NOT_CONVERGED (> 0): the output was written (best iterate) but
 * the requested tolerance was not reached. dfl_last_error() returns a
 * thread-local message for the last failing call. No C++ exception crosses
 * this interface.
 */
#ifndef DFL_H
#define DFL_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dfl_ctx dfl_ctx;

typedef enum {
    DFL_OK = 0,
    DFL_NOT_CONVERGED = 1, /* output written, tolerance not met */
    DFL_EINVAL = -1,       /* bad argument: shape, null pointer, range */
    DFL_ENOMEM = -2,       /* device allocation failed */
    DFL_EHIP = -3,         /* HIP runtime error */
    DFL_ESINGULAR = -4,    /* block Gram-Schmidt lost rank, or a singular solve */
    DFL_ENONFINITE = -5,   /* NaN or Inf in an input or a reduction */
    DFL_ESTATE = -6        /* call out of order (e.g. projection before dfl_setup) */
} dfl_status;

typedef enum { DFL_F64 = 0, DFL_F32 = 1, DFL_BF16 = 2 } dfl_prec;

/* which projector deflate_project applies (section 3.1) */
typedef enum {
    DFL_PROJ_PL = 0,     /* P_L y = y - D Phi A^-1 Phi^+ y, eq. (3.3) */
    DFL_PROJ_PR = 1,     /* P_R y = y - Phi A^-1 Phi^+ D y, eq. (3.4) */
    DFL_PROJ_P = 2,      /* P y = Phi Phi^+ y, eqs. (3.1)/(4.1) */
    DFL_PROJ_COARSE = 3  /* Phi A^-1 Phi^+ y, the coarse term of eq. (3.10) */
} dfl_proj;

/* which solver solve() runs */
typedef enum {
    DFL_SOLVER_GCR = 0,         /* plain GCR on D psi = eta */
    DFL_SOLVER_SAP_GCR = 1,     /* GCR right-preconditioned by M_sap */
    DFL_SOLVER_DFL_SAP_GCR = 2  /* deflated + SAP-preconditioned, eq. (6.2) */
} dfl_solver;

typedef struct {
    int dims[4];        /* L0..L3, x0 slowest; each a multiple of both block shapes;
                           volume a multiple of 64 and at most 2^22 sites */
    int sap_block[4];   /* Schwarz blocks; dims[mu]/sap_block[mu] even and >= 2 */
    int dfl_block[4];   /* deflation blocks; dims[mu]/dfl_block[mu] even and >= 2 */
    int Ns;             /* deflation fields per block, 1 <= Ns <= 12*|dfl_block| (and <= 64) */
    int ncy;            /* SAP cycles per application (>= 1) */
    int nmr;            /* minimal-residual steps per block solve (>= 1) */
    int nkv;            /* Krylov vectors before a GCR restart (1..64); with inexact
                           inner projections a cycle also ends once its residue fell
                           by 10*little_tol_in */
    int n_inviter;      /* inverse-iteration steps in dfl_setup (>= 0) */
    int maxiter;        /* outer GCR iteration limit */
    int nrhs_max;       /* largest nrhs any call will pass (1..16); field workspaces
                           scale with it */
    int little_nkv;     /* Krylov vectors of the little GCR (1..32) */
    int little_maxiter; /* little GCR iteration limit */
    dfl_solver solver;  /* variant run by solve() */
    double m0;          /* bare mass of D */
    double m0_setup;    /* bare mass used by the inverse iteration of dfl_setup */
    double tol;         /* solve() stops at ||eta - D psi|| <= tol ||eta|| */
    double little_tol_in;  /* little-solve tolerance inside GCR cycles (appendix A.5) */
    double little_tol_out; /* little-solve tolerance at restarts and the final step */
    dfl_prec link_prec;    /* link storage of the SAP block solves: F64, F32 or BF16 two-row */
    dfl_prec sap_prec;     /* arithmetic of the SAP block solves: F64 or F32 */
    dfl_prec little_prec;  /* arithmetic of the little solves inside cycles: F64 or F32 */
    int little_grid;       /* workgroups of the little solver (0: a quarter of the block
                              count); clamped to the block count, to 256 and to the
                              number of workgroups the device holds at once */
    int little_adapt;      /* 1: inside a cycle, relax the little-solve tolerance in
                              proportion to the fall of the residue (appendix A.5) */
    int little_eo;         /* 1: little solves (single-source and batched) run GCR on the
                              even-odd reduced system (appendix A.2), falling back to A
                              when a diagonal block is not safely invertible */
    int little_gdefl;      /* global-mode deflation of the even-odd little system
                              (appendix A.3; with little_eo and Ns <= 32) by the
                              even-block parts of the global fields the subspace was built
                              from, i.e. the inverse-iteration fields before block
                              orthonormalisation. 0: off; 1: minimal-residual form (the
                              residue kept orthogonal to A_hat Z); 2: section 3's oblique
                              projectors with the Ns x Ns "little little" operator
                              Z^+ A_hat Z inverted exactly */
    double csw;            /* coefficient of the O(a)-improvement (clover) term of section
                              2.1, csw (i/4) sum_{mu,nu} sigma_{mu nu} Fhat_{mu nu}(x), Fhat
                              from the four plaquettes around x; 0: plain Wilson */
    int antiperiodic;      /* 1: antiperiodic quark boundary condition in direction 0
                              (time), 0: periodic; space is always periodic */
    int n_boot;            /* 0..n_inviter: the last n_boot inverse-iteration steps of
                              dfl_setup are bootstrapped (section 5.3): the fields of the
                              previous step span a subspace that deflates the approximate
                              solve, psi <- P_R M_sap P_L psi + Phi A^-1 Phi^+ psi (eqs. (3.10),
                              (3.11)), little solves to little_tol_in in little_prec;
                              needs 2 Ns more FP64 fields of device memory */
} dfl_params;

typedef struct {
    int status;          /* dfl_status of the solve */
    int n_gcr;           /* outer GCR iterations (Krylov vectors generated) */
    int n_restarts;      /* outer restarts */
    int n_little;        /* little GCR iterations summed over all little solves */
    int n_little_solves; /* number of little solves */
    double rel_residual; /* ||eta - D psi|| / ||eta||, recomputed in FP64 at the end */
    double t_solve;      /* seconds from entry to return */
    double t_setup;      /* seconds of the last dfl_setup on this context (entry to return;
                            0 before the first) */
    double t_sap;        /* kernel seconds of this solve in the Schwarz sweeps, the stencil, */
    double t_dirac;      /* the restriction and prolongation and the little solves, from the */
    double t_proj;       /* library's event timers while dfl_profile_enable(ctx, 1) is on; */
    double t_little;     /* -1 when it is off (the timers cost a few us per launch) */
} dfl_info;

/* Fill *p with defaults: 4^4 blocks, Ns = 20, ncy = 5, nmr = 4, nkv = 16,
 * n_inviter = 3, maxiter = 1000, tol = 1e-10, little tolerances 1e-6/1e-12
 * with adapted precision, even-odd little solves and their global-mode
 * deflation on, all precisions F64,
 * solver DFL_SAP_GCR; dims are left zero. */
void dfl_default_params(dfl_params *p);

/* Create a context for the lattice and parameters in *p on the current HIP
 * device; hip_stream is a hipStream_t (NULL: the null stream). Allocates the
 * gauge storage and solver workspaces for nrhs_max right-hand sides.
 * Errors: DFL_EINVAL (shapes, see dfl_params), DFL_ENOMEM, DFL_EHIP. */
int dfl_create(dfl_ctx **ctx, const dfl_params *p, void *hip_stream);

/* Release the context and every buffer it owns. NULL is a no-op. */
int dfl_destroy(dfl_ctx *ctx);

/* Change the bare mass m0 of D (and of the little operator, which shifts by
 * (m0' - m0) times the identity since the basis is orthonormal). */
int dfl_set_mass(dfl_ctx *ctx, double m0);

/* Size in bytes of one native quark field of precision prec (F64 or F32). */
long long dfl_field_bytes(const dfl_ctx *ctx, dfl_prec prec);

/* Number of deflation blocks Nb (the little vector has Nb*Ns entries). */
int dfl_num_blocks(const dfl_ctx *ctx);

/* Load the gauge field U (canonical complex128 [V][4][3][3], device) and
 * derive the internal copies, two rows per SU(3) matrix (the third is
 * rebuilt as conj(row0 x row1) where a link is used): FP64 for D, FP32 and
 * BF16 for the SAP block solves. Synchronises. DFL_EINVAL (and no gauge
 * field) if some link's third row differs from conj(row0 x row1) by more than
 * 1e-12 relative, i.e. the links are not SU(3). Invalidates a previously
 * built deflation subspace. */
int dfl_set_gauge(dfl_ctx *ctx, const double *U_canon_dev);

/* Canonical complex128 [nrhs][V][12] (device) <-> native fields of precision
 * prec (F64 or F32; FP32 rounds to nearest). */
int dfl_pack(dfl_ctx *ctx, const double *canon_dev, void *native_dev, int nrhs, dfl_prec prec);
int dfl_unpack(dfl_ctx *ctx, const void *native_dev, double *canon_dev, int nrhs, dfl_prec prec);

/* out = D psi for nrhs native fields (eq. (3.9)'s operator). prec F64 uses
 * the FP64 full links; F32 uses FP32 arithmetic on FP32 fields with the links
 * in the context's SAP link precision (F32 or BF16 two-row; F64 links are
 * rounded to F32 two-row). psi and out must not overlap. */
int dirac_apply(dfl_ctx *ctx, const void *psi_dev, void *out_dev, int nrhs, dfl_prec prec);

/* psi = M_sap rho, the Schwarz alternating procedure of eq. (6.2) (and the
 * relaxation of eq. (5.1)): ncy cycles; in each, every block of colour 0 and
 * then of colour 1 adds nmr minimal-residual steps for D_Lambda x = (rho - D psi)|_Lambda.
 * rho and psi are native FP64 fields; the block solves run in sap_prec with
 * links in link_prec. psi and rho must not overlap. */
int sap_precond(dfl_ctx *ctx, const void *rho_dev, void *psi_dev, int nrhs);

/* Build the deflation subspace (section 5.3, eq. (4.2), eq. (A.1)): the Ns
 * native FP64 start fields init_dev (random; the caller draws them) are
 * normalised, relaxed by n_inviter steps psi_l <- M_sap psi_l / ||.|| at
 * m0_setup, restricted to the deflation blocks and orthonormalised by
 * Gram-Schmidt in the order l = 1..Ns; then the little operator A is
 * assembled at the current m0. n_init must equal Ns. init_dev is not modified.
 * Synchronises. Errors: DFL_ESINGULAR if a block loses rank. */
int dfl_setup(dfl_ctx *ctx, const void *init_dev, int n_init);

/* Copy the orthonormal basis out: Ns native FP64 fields whose restriction to
 * block Lambda is phi^Lambda_l (section 4.1). */
int dfl_get_basis(dfl_ctx *ctx, void *phi_dev);

/* Copy the little operator out, complex128 [Nb][9][Ns][Ns] (device): index 0
 * the block itself, 1 + 2*mu the block Lambda + mu_hat, 2 + 2*mu the block
 * Lambda - mu_hat, entry [k][l] = (phi^Lambda_k, D phi^Lambda'_l) (eq. (A.1)),
 * each neighbour term holding only the hops across that one face. */
int dfl_get_little(dfl_ctx *ctx, double *A_dev);

/* w = A v with the little Dirac operator (eqs. (3.2)/(A.1)) for nrhs native
 * little vectors of precision prec (F64 or F32), back to back. One launch for
 * all nrhs; F32 with nrhs > 1 runs as a batched complex GEMM on the matrix
 * cores (16 right-hand sides per pass). */
int little_dirac_apply(dfl_ctx *ctx, const void *v_dev, void *w_dev, int nrhs, dfl_prec prec);

/* Solve A v = w (eq. (6.1)) by GCR to ||w - A v|| <= tol ||w|| in FP64
 * (native FP64 little vectors). Returns DFL_NOT_CONVERGED if little_maxiter
 * is reached. iters (may be NULL) receives the iteration count. */
int little_solve(dfl_ctx *ctx, const void *w_dev, void *v_dev, double tol, int *iters);

/* out = (projector which) in, for native FP64 fields (section 3.1); the little
 * solves run to little_tol_out in FP64. in and out must not overlap. */
int deflate_project(dfl_ctx *ctx, dfl_proj which, const void *in_dev, void *out_dev, int nrhs);

/* Run the GCR steps of solve() as HIP graphs (on != 0) or as direct
 * launches (0, the default). With graphs on, the launch sequence of each
 * Krylov step (Schwarz preconditioner, stencil, deflation projector with its
 * little solve, Gram-Schmidt) is captured once per step index and number of
 * sources and replayed on later steps and solves; results are identical to
 * direct launches. The captured little solve is an ordinary kernel node whose
 * grid of at most one workgroup per compute unit is resident when nothing
 * else runs on the device. Graphs are dropped when the mass changes. Capture
 * and replay run on a stream the context creates, ordered against the
 * context's stream by events. Synchronises. */
int dfl_use_graphs(dfl_ctx *ctx, int on);

/* Number of graph replays since the context was created (-1 for NULL). */
long long dfl_graph_replays(const dfl_ctx *ctx);

/* Solve D psi = eta for nrhs native FP64 sources to ||eta - D psi|| <= tol ||eta||
 * with the solver chosen in the parameters (section 6 for DFL_SAP_GCR:
 * flexible GCR on eq. (6.2), restarts recomputing the residual in FP64
 * (appendix A.5), final solution by eq. (3.10)). psi is overwritten (the start
 * vector is zero). The nrhs sources are solved together: every stencil,
 * Schwarz, projection and little-solve launch covers all of them, while each
 * keeps its own Krylov coefficients and stops on its own residual.
 * Synchronises; info (may be NULL) points to nrhs records, one per source
 * (little-solve counts and t_solve are those of the whole call). Returns
 * DFL_NOT_CONVERGED if some source reached maxiter. */
int solve(dfl_ctx *ctx, const void *eta_dev, void *psi_dev, int nrhs, dfl_info *info);

/* Relative residue norms of the last outer GCR run (the initial one, then one
 * per Krylov step, as updated by the recursion), the last right-hand side of
 * the last solve(). Copies min(count, max) values to out (host memory) and
 * returns count, or -1 for a null context or bad arguments. Host-only. */
int dfl_residual_history(const dfl_ctx *ctx, double *out, int max);

/* Kernel-class timers. When enabled, the context records a pair of HIP
 * events on its stream around every launch of the classes below (a small
 * overhead per launch); dfl_profile_read synchronises and returns the summed
 * seconds and launch counts per class since the last reset, then resets.
 * Classes: */
enum {
    DFL_PROF_SAP = 0,      /* Schwarz colour sweeps of the solvers and sap_precond (one launch per colour and cycle) */
    DFL_PROF_DIRAC = 1,    /* full-lattice Dirac operator inside the solvers and dirac_apply */
    DFL_PROF_LITTLE = 2,   /* little GCR (one cooperative launch per little solve) */
    DFL_PROF_PROJECT = 3,  /* block restriction and prolongation */
    DFL_PROF_SETUP = 4,    /* block Gram-Schmidt, little-operator assembly and its even-odd and global-mode preparation */
    DFL_PROF_SETUP_SAP = 5, /* Schwarz sweeps of the inverse iteration (all Ns fields per launch) */
    DFL_PROF_NCLASS = 6
};
int dfl_profile_enable(dfl_ctx *ctx, int on);
/* seconds[DFL_PROF_NCLASS], launches[DFL_PROF_NCLASS] (host memory); little_iters
 * (may be NULL) receives the little GCR iterations of the same launches. */
int dfl_profile_read(dfl_ctx *ctx, double *seconds, long long *launches, long long *little_iters);

/* Message of the last failing call on this thread ("" if none). */
const char *dfl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DFL_H */
