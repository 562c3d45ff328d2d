"""Benchmark of the deflated SAP-GCR solver on one MI355X.

Workload (one "step"): the 16^4 lattice at two gauge roughnesses (eps 0.4 and
0.6, seeds 2001/2002); per gauge field one subspace setup (Ns = 20 fields,
3 inverse-iteration steps, 4^4 blocks) reused for the three masses
m0 = -0.2, -0.3, -0.35 (the subspace is generated once per gauge field and
used at all valence masses), each solved to ||eta - D psi|| <= 1e-10 ||eta||
with FP64 flexible GCR, FP32 Schwarz block solves (4^4 blocks, 5 cycles,
4 MR steps) and FP64 little solves. value = solves per second over the
whole step (setups included).

Besides the step the run reports:
* dirac_apply GFLOP/s and algorithmic GB/s on 64 x 32^3 (FP64 full links,
  FP32 and BF16 two-row links), a working set well above the 256 MB MALL;
* the dominant kernel's roofline, timed with HIP events on the library stream;
* undeflated SAP+GCR and plain GCR on the same fields (iterations, seconds);
* the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector
FP64_VECTOR_PEAK_TFLOPS = 78.6
FLOPS_PER_SITE = 1368            # Wilson stencil, per site per right-hand side
BYTES_PER_SITE = {"f64": 960, "f32_tworow": 384, "bf16_tworow": 288}

DIMS = (16, 16, 16, 16)
BLOCK = (4, 4, 4, 4)
FIELDS = [(0.4, 2001), (0.6, 2002)]
MASSES = [-0.2, -0.3, -0.35]
NS, NCY, NMR, NKV, NINV = 20, 5, 4, 16, 3
TOL = 1e-10


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_inputs():
    import latgen
    fields = []
    for eps, seed in FIELDS:
        U = latgen.make_links(DIMS, eps, seed)
        eta = latgen.make_source(DIMS, seed + 100)
        init = latgen.make_init_fields(DIMS, NS, seed + 200)
        fields.append(dict(eps=eps, seed=seed, U=U, eta=eta, init=init))
    return fields


def solver_params(**kw):
    from paper_0706_2298_amd import F32, F64
    p = dict(dfl_block=BLOCK, sap_block=BLOCK, Ns=NS, ncy=NCY, nmr=NMR, nkv=NKV, n_inviter=NINV,
             m0=MASSES[0], m0_setup=min(MASSES), tol=TOL, sap_prec=F32, link_prec=F32, little_prec=F64,
             little_tol_in=1e-6, little_tol_out=1e-12, maxiter=4000)
    p.update(kw)
    return p


def run_step(ctxs, stats=None):
    for c in ctxs:
        c["S"].setup(c["init"])
        for m in MASSES:
            c["S"].set_mass(m)
            _, info = c["S"].solve(c["eta"])
            if stats is not None:
                stats.append(dict(eps=c["eps"], m0=m, **info.as_dict()))
            if info.status != 0:
                raise RuntimeError(f"solve failed: {info.as_dict()}")


def time_events(torch, fn, reps):
    """Average duration of fn() in seconds, HIP events on the current stream."""
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    e0.record(st)
    for _ in range(reps):
        fn()
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def dirac_rates(torch):
    """dirac_apply on 64 x 32^3: FP64 full links, FP32 and BF16 two-row links."""
    import latgen
    from paper_0706_2298_amd import BF16, F32, F64, Solver
    dims = (64, 32, 32, 32)
    V = int(np.prod(dims))
    U = latgen.make_links(dims, 0.4, 4101)
    psi = latgen.make_source(dims, 4102)
    out = {}
    for name, lp, prec in [("f64", F64, F64), ("f32_tworow", F32, F32), ("bf16_tworow", BF16, F32)]:
        sp = F64 if lp == F64 else F32
        S = Solver(dims, Ns=1, nkv=1, little_nkv=1, m0=-0.2, link_prec=lp, sap_prec=sp)
        S.set_gauge(U)
        x = S.pack(psi, prec=prec)
        y = S.field(1, prec)
        from paper_0706_2298_amd import binding
        t = time_events(torch, lambda: binding.dirac_apply(S.ctx, x, y, 1, prec), 40)
        out[name] = dict(ms=t * 1e3, gflops=FLOPS_PER_SITE * V / t / 1e9,
                         gbs=BYTES_PER_SITE[name] * V / t / 1e9,
                         frac_hbm=BYTES_PER_SITE[name] * V / t / 1e9 / HBM_PEAK_GBS)
        S.close()
        del x, y
    torch.cuda.empty_cache()
    return out


def undeflated(torch, fields):
    from paper_0706_2298_amd import SOLVER_GCR, SOLVER_SAP_GCR, Solver
    rows = []
    for f in fields:
        for solver, nkv, name in [(SOLVER_SAP_GCR, 32, "sap_gcr"), (SOLVER_GCR, 32, "gcr_f64")]:
            S = Solver(DIMS, **solver_params(solver=solver, nkv=nkv, Ns=1, maxiter=20000))
            S.set_gauge(f["U"])
            eta = S.pack(f["eta"])
            for m in MASSES:
                S.set_mass(m)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, info = S.solve(eta)
                torch.cuda.synchronize()
                rows.append(dict(solver=name, eps=f["eps"], m0=m, n_gcr=info.n_gcr, status=info.status,
                                 rel_residual=info.rel_residual, seconds=time.perf_counter() - t0))
            S.close()
    return rows


def cpu_baseline(fields, stats):
    """The FP64 oracle on a bounded sample of the step, scaled to solves/s.

    Sample: for the eps = 0.4 field, one Schwarz application, one inverse-
    iteration normalisation, the block Gram-Schmidt and little-operator
    assembly on the 20 start fields (without relaxation), and two iterations
    of the deflated GCR at m0 = -0.3; the step's cost is then the GPU run's
    own operation counts (setup SAP applications, GCR iterations, restarts)
    times these unit costs.
    """
    import oracle
    f = fields[0]
    U, eta, init = f["U"], f["eta"], f["init"]
    m0 = -0.3
    t0 = time.perf_counter()
    oracle.sap(U, eta, m0, DIMS, BLOCK, NCY, NMR)
    t_sap = time.perf_counter() - t0
    t0 = time.perf_counter()
    Phi = oracle.block_gram_schmidt(init, DIMS, BLOCK)
    t_gs = time.perf_counter() - t0
    t0 = time.perf_counter()
    A = oracle.little_operator(U, Phi, m0, DIMS, BLOCK)
    t_little_op = time.perf_counter() - t0
    dfl = oracle.Deflation(U, Phi, A, m0, DIMS, BLOCK)
    t0 = time.perf_counter()
    _, it, _ = oracle.solve(U, eta, m0, DIMS, sap_block=BLOCK, ncy=NCY, nmr=NMR, dfl=dfl, tol=1e-30, maxiter=2)
    t_two = time.perf_counter() - t0
    sample_s = t_sap + t_gs + t_little_op + t_two
    # per-iteration cost (the two-iteration solve also pays one initial projection, one restart and the final step)
    t_iter = t_two / 2.0
    n_setup_sap = len(fields) * NS * NINV
    n_iter = sum(s["n_gcr"] for s in stats)
    est = n_setup_sap * t_sap + len(fields) * (t_gs + t_little_op) + n_iter * t_iter
    n_solves = len(stats)
    return dict(value=n_solves / est, unit="solves/s", cores=oracle.num_threads(), kind="oracle",
                sample=(f"16^4 eps=0.4: 1 SAP application ({t_sap:.2f}s), block GS + little operator on 20 fields "
                        f"({t_gs + t_little_op:.2f}s), 2 deflated GCR iterations ({t_two:.2f}s); scaled by the "
                        f"step's {n_setup_sap} setup SAP applications and {n_iter} GCR iterations "
                        f"-> {est:.1f}s per step of {n_solves} solves"),
                sample_seconds=sample_s)


def dominant_kernel_roofline(torch, ctx_entry):
    """SAP colour sweep (FP32, 4^4 blocks) timed alone with HIP events."""
    from paper_0706_2298_amd import binding
    S = ctx_entry["S"]
    rho = ctx_entry["eta"]
    psi = S.field(1)
    t_sap = time_events(torch, lambda: binding.sap_precond(S.ctx, rho, psi, 1), 20)
    return t_sap


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dirac", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_0706_2298_amd import Solver
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(3)
    torch.cuda.set_device(0)

    log("generating inputs")
    fields = make_inputs()
    ctxs = []
    for f in fields:
        S = Solver(DIMS, **solver_params())
        S.set_gauge(f["U"])
        ctxs.append(dict(S=S, eps=f["eps"], eta=S.pack(f["eta"]), init=S.pack(f["init"])))
    torch.cuda.synchronize()

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        run_step(ctxs)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    stats = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        run_step(ctxs, stats if k == 0 else None)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    n_solves = len(FIELDS) * len(MASSES)
    log(f"step {dt * 1e3:.1f} ms")

    result = {
        "metric": "dirac_apply GFLOP/s + HBM GB/s; time-to-solution @ rel. residual 1e-10",
        "value": n_solves / dt,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "16^4 DFL+SAP+GCR, eps {0.4,0.6}, m0 {-0.2,-0.3,-0.35}, Ns 20, 4^4 blocks, "
                               "FP64 GCR + FP32 SAP, tol 1e-10",
                   "lattice": list(DIMS), "Ns": NS, "n_inviter": NINV, "ncy": NCY, "nmr": NMR, "nkv": NKV,
                   "solves_per_step": n_solves},
        "solves": stats,
    }
    t_sap = dominant_kernel_roofline(torch, ctxs[0])
    result["sap_precond_ms"] = t_sap * 1e3
    for c in ctxs:
        c["S"].close()
    ctxs.clear()
    torch.cuda.empty_cache()

    if not args.no_dirac:
        log("dirac_apply on 64x32^3")
        result["dirac_apply"] = dirac_rates(torch)
    if not args.no_compare:
        log("undeflated comparisons")
        result["undeflated"] = undeflated(torch, fields)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(fields, stats)
    result["host"] = {"cpu": platform.processor() or platform.machine(), "nproc": os.cpu_count()}
    print(json.dumps(result))


if __name__ == "__main__":
    main()
