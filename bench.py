"""Benchmark of the deflated SAP-GCR solver on one MI355X.

Headline workload (one "step"): the 64 x 32^3 lattice (2,097,152 sites) with
the link field U = exp(i 0.5 H) of seed 5100 and a Gaussian source (seed
5200), bare mass m0 = -0.56 (near the critical mass of this gauge
roughness). A step is one subspace setup (Ns = 24 random start fields, seed
5300, 3 inverse-iteration steps, 4^4 deflation blocks, block Gram-Schmidt and
little-operator assembly) followed by one solve to ||eta - D psi|| <= 1e-10
||eta|| with FP64 flexible GCR (16 Krylov vectors), FP32 Schwarz block solves
(4^4 blocks, 5 cycles, 4 MR steps, FP32 two-row links), FP32 little solves
inside GCR cycles and FP64 ones (1e-12) at restarts and for the final
correction. value = steps per second (one setup plus one solve each); the
setup and solve times are reported apart. All inputs are resident in HBM
before the timed region; the true residual of every timed solve is recomputed
in FP64.

Also reported (outside the timed region):
* the dominant kernel's roofline: one extra step with the library's
  kernel-class event timers on; algorithmic flops or bytes per launch over
  the measured launch duration, with the rocprofv3 counter traffic when the
  committed counter summary matches the kernel source;
* dirac_apply GFLOP/s and GB/s on 64 x 32^3 (FP64, FP32 and BF16 two-row
  links) and with 12 sources on 48 x 24^3;
* on the headline field: undeflated SAP+GCR, plain FP64 GCR, the deflated
  solver with FP64 inner little solves, with the oblique global-mode deflation
  of the little system (appendix A.3 as written) and with a bootstrapped setup
  (section 5.3);
* 32 x 16^3 in mixed precision (BF16 two-row links; Schwarz block shape and
  little-solver grid from the autotuner) against the all-FP64 deflated solver and plain FP64 GCR, with
  errors against FP64 references;
* 12 point sources on 48 x 24^3 and 6 on 32 x 16^3 (Ns = 24) as one batch per
  lattice with graph replay, against one-by-one solves and plain FP64 GCR;
* the learned start fields: the network trained on 16^4 fields (eps 0.5),
  then on 5 held-out 64 x 32^3 fields the setup and solve times against
  random start fields and plain FP64 GCR, with the forward pass in FP32 and
  with BF16 operands;
* the 16^4 workload (two gauge fields x three masses) against undeflated
  solvers;
* the FP64 CPU oracle timed on a bounded sample, scaled to the headline step.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_NONPACKED_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12  # 78.6: one (non-packed) FP32 FMA per lane and cycle
FLOPS_PER_SITE = 1368            # Wilson stencil per site per right-hand side (1320 hop + 48 diagonal)
# links are stored as two rows of the SU(3) matrix in every precision (the third row is rebuilt)
BYTES_PER_SITE = {"f64_tworow": 768, "f32_tworow": 384, "bf16_tworow": 288}

# headline workload
DIMS = (64, 32, 32, 32)
BLOCK = (4, 4, 4, 4)
EPS, SEED, M0 = 0.5, 5100, -0.56
NS, NCY, NMR, NKV, NINV = 24, 5, 4, 16, 3
TOL = 1e-10
V = int(np.prod(DIMS))
NB = V // int(np.prod(BLOCK))

# the 16^4 workload
C2_DIMS = (16, 16, 16, 16)
C2_FIELDS = [(0.4, 2001), (0.6, 2002)]
C2_MASSES = [-0.2, -0.3, -0.35]


def sap_flops_per_site(nmr):
    # residual rho - D psi (1368 + 24), nmr MR steps of D_Lambda (1368) plus
    # (q,r), (q,q), x += a r, r -= a q (96 + 48 + 96 + 96), and psi += x (24)
    return 1368 + 24 + nmr * (1368 + 336) + 24


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def params(**kw):
    from paper_0706_2298_amd import F32, F64
    p = dict(dfl_block=BLOCK, sap_block=BLOCK, Ns=NS, ncy=NCY, nmr=NMR, nkv=NKV, n_inviter=NINV,
             m0=M0, m0_setup=M0, tol=TOL, sap_prec=F32, link_prec=F32, little_prec=F32,
             little_tol_in=1e-6, little_tol_out=1e-12, maxiter=4000)
    p.update(kw)
    return p


def timed(torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


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


def headline_inputs():
    import latgen
    U = latgen.make_links(DIMS, EPS, SEED)
    eta = latgen.make_source(DIMS, SEED + 100)
    init = latgen.make_init_fields(DIMS, NS, SEED + 200)
    return U, eta, init


def step(torch, S, eta, init):
    """One setup + one solve; (t_setup, t_solve, info)."""
    _, t_setup = timed(torch, lambda: S.setup(init))
    (_, info), t_solve = timed(torch, lambda: S.solve(eta))
    if info.status != 0:
        raise RuntimeError(f"solve failed: {info.as_dict()}")
    return t_setup, t_solve, info


def profiled(S, fn):
    """Run fn with the library's kernel-class timers on; {class: (s, launches)} and little iterations."""
    from paper_0706_2298_amd import binding
    binding.dfl_profile_read(S.ctx)
    binding.dfl_profile_enable(S.ctx, True)
    fn()
    p = binding.dfl_profile_read(S.ctx)
    binding.dfl_profile_enable(S.ctx, False)
    return p


def source_digest(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_0706_2298_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {"sap": ("sap.hip", "hop.h", "common.h"), "setup_sap": ("sap.hip", "hop.h", "common.h"),
                  "little": ("little.hip", "common.h"), "dirac": ("dirac.hip", "hop.h", "common.h"),
                  "project": ("dfl.hip", "common.h")}


def counter_traffic(name, digest_of):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    profiles/<name>_counters.md, if it was taken on the current source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{name}_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"source digest:\s*([0-9a-f]+)", txt)
    b = re.search(r"hbm bytes per launch:\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != source_digest(*KERNEL_SOURCES[digest_of]):
        return None
    return float(b.group(1))


def roofline(prof):
    """Roofline object for the kernel class that took the most time in the profiled step
    (the setup's block Gram-Schmidt and assembly class is a mix of kernels and is left out)."""
    cls = max(("sap", "setup_sap", "little", "dirac", "project"), key=lambda k: prof[k][0])
    sec, n = prof[cls]
    dur = sec / max(n, 1)
    half = V // 2   # one colour sweep visits half the sites
    if cls in ("sap", "setup_sap"):
        nf = 1 if cls == "sap" else NS
        flops = sap_flops_per_site(NMR) * half * nf
        ach = flops / dur / 1e12
        kern = ("k_sap_rl<Links32, 4^4> (Schwarz colour sweep of one field, FP32, one lane per site)"
                if cls == "sap" else
                f"k_sap_rl<Links32, 4^4> (Schwarz colour sweep of the {NS} inverse-iteration fields, FP32)")
        r = dict(kernel=kern, bound="alu", achieved=ach, peak=FP32_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                 frac=ach / FP32_VECTOR_PEAK_TFLOPS,
                 per_launch=f"{flops:.4g} flop = {sap_flops_per_site(NMR)} flop/site x {half} sites x {nf} fields",
                 # the library is built without packed FP32 instructions: one FP32 FMA per lane and cycle,
                 # 256 CUs x 64 lanes x 2 flop x 2.4 GHz
                 peak_nonpacked=FP32_NONPACKED_PEAK_TFLOPS, frac_nonpacked=ach / FP32_NONPACKED_PEAK_TFLOPS)
    elif cls == "little":
        it = prof["little_iterations"] / max(n, 1)
        # even-odd step: the eight neighbour blocks of D^-1 A over all blocks
        # (two half-applies) in FP32, plus four vectors
        per_it = NB * (8 * NS * NS * 8 + 4 * NS * 8)
        byts = per_it * it
        ach = byts / dur / 1e9
        r = dict(kernel="k_little_gcr<float, true> (even-odd little GCR, FP32, one launch per little solve)",
                 bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                 per_launch=f"{byts:.4g} B = {it:.1f} iterations x {per_it} B (D^-1 A blocks + 4 vectors, FP32)")
    elif cls == "dirac":
        byts = BYTES_PER_SITE["f64_tworow"] * V
        ach = byts / dur / 1e9
        r = dict(kernel="k_dirac_blk<double>", bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                 frac=ach / HBM_PEAK_GBS, per_launch=f"{byts} B = 768 B/site x {V}")
    else:
        byts = 192 * (NS + 1) * V
        ach = byts / dur / 1e9
        r = dict(kernel="k_restrict_kg / k_prolong (FP64)", bound="hbm", achieved=ach, peak=HBM_PEAK_GBS,
                 unit="GB/s", frac=ach / HBM_PEAK_GBS,
                 per_launch=f"{byts} B = (Ns + 1) fields x 192 B/site x {V}")
    r["class"] = cls
    r["avg_launch_us"] = dur * 1e6
    r["launches_per_step"] = n
    r["traffic"] = counter_traffic(cls, cls)
    return r


def dirac_rates(torch):
    """dirac_apply on 64 x 32^3: FP64 arithmetic with FP64 two-row links, FP32 with FP32 and BF16
    two-row links (a working set well above the 256 MB MALL), with the counter traffic."""
    import latgen
    from paper_0706_2298_amd import BF16, F32, F64, Solver, binding
    U = latgen.make_links(DIMS, 0.4, 4101)
    psi = latgen.make_source(DIMS, 4102)
    out = {}
    for name, lp, prec in [("f64_tworow", F64, F64), ("f32_tworow", F32, F32), ("bf16_tworow", BF16, F32)]:
        sp = F64 if lp == F64 else F32
        S = Solver(DIMS, Ns=1, nkv=1, little_nkv=1, m0=-0.2, link_prec=lp, sap_prec=sp)
        S.set_gauge(U)
        x = S.pack(psi, prec=prec)
        y = S.field(1, prec)
        t = time_events(torch, lambda: binding.dirac_apply(S.ctx, x, y, 1, prec), 40)
        gbs = BYTES_PER_SITE[name] * V / t / 1e9
        out[name] = dict(us=t * 1e6, gflops=FLOPS_PER_SITE * V / t / 1e9, gbs=gbs, frac_hbm=gbs / HBM_PEAK_GBS)
        S.close()
        del x, y
    torch.cuda.empty_cache()
    # achievable HBM rate for reference: a device-to-device copy of one FP64 64 x 32^3 field (402 MB);
    # each stencil rate is also given as a fraction of it
    a = torch.ones(24 * V, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    t = time_events(torch, lambda: b.copy_(a), 20)
    out["copy_gbs"] = 2 * a.numel() * 8 / t / 1e9
    for name in BYTES_PER_SITE:
        out[name]["frac_copy"] = out[name]["gbs"] / out["copy_gbs"]
    del a, b
    # 12 fields in one launch on 48 x 24^3 against one field (per field and site: FP64 384 B of
    # spinors, FP32 192 B; the two-row links, 384 / 192 B per site, once per launch)
    dims12 = (48, 24, 24, 24)
    v12 = int(np.prod(dims12))
    U12 = latgen.make_links(dims12, 0.4, 4001)
    src = latgen.random_field(dims12, 4003, n=12)
    multi = {}
    for name, lp, prec, sb, lb in [("f64", F64, F64, 384, 384), ("f32", F32, F32, 192, 192)]:
        S = Solver(dims12, Ns=1, nkv=1, little_nkv=1, m0=-0.3, link_prec=lp, sap_prec=prec, nrhs_max=12)
        S.set_gauge(U12)
        x = S.pack(src, prec=prec)
        y = S.field(12, prec)
        x1 = S.pack(src[0], prec=prec)
        y1 = S.field(1, prec)
        t12 = time_events(torch, lambda: binding.dirac_apply(S.ctx, x, y, 12, prec), 10)
        t1 = time_events(torch, lambda: binding.dirac_apply(S.ctx, x1, y1, 1, prec), 20)
        gbs = (12 * sb + lb) * v12 / t12 / 1e9
        multi[name] = dict(us_12=t12 * 1e6, us_1=t1 * 1e6, per_field_speedup=12 * t1 / t12,
                           gflops_12=FLOPS_PER_SITE * v12 * 12 / t12 / 1e9, gbs_12=gbs,
                           frac_hbm_12=gbs / HBM_PEAK_GBS)
        S.close()
        del x, y, x1, y1
        torch.cuda.empty_cache()
    out["multi_field_48x24"] = multi
    for name, summary in [("f64_tworow", "dirac64"), ("f32_tworow", "dirac32"), ("bf16_tworow", "diracbf16")]:
        tr = counter_traffic(summary, "dirac")
        if tr is not None:
            out[name]["counter_bytes_per_launch"] = tr
            out[name]["counter_gbs"] = tr / (out[name]["us"] * 1e-6) / 1e9
    return dict(lattice=list(DIMS), bytes_per_site=BYTES_PER_SITE, flops_per_site=FLOPS_PER_SITE, **out)


def comparisons(torch, U, eta, init):
    """Other solvers and variants on the headline field (time to solution, iterations)."""
    from paper_0706_2298_amd import F64, SOLVER_GCR, SOLVER_SAP_GCR, Solver
    rows = {}
    for name, kw in [("sap_gcr", dict(solver=SOLVER_SAP_GCR, nkv=32, Ns=1, maxiter=20000)),
                     ("gcr_f64", dict(solver=SOLVER_GCR, nkv=32, Ns=1, maxiter=20000))]:
        S = Solver(DIMS, **params(**kw))
        S.set_gauge(U)
        ed = S.pack(eta)
        (_, info), t = timed(torch, lambda: S.solve(ed))
        rows[name] = dict(t_solve=t, n_gcr=info.n_gcr, status=info.status, rel_residual=info.rel_residual)
        S.close()
        del ed
        torch.cuda.empty_cache()
        log(f"{name}: {info.n_gcr} iterations, {t:.3f} s")
    for name, kw in [("dfl_little_f64", dict(little_prec=F64)),
                     ("dfl_oblique_little_deflation", dict(little_gdefl=2)),
                     ("dfl_bootstrap_1", dict(n_boot=1)),
                     ("dfl_bootstrap_2_ninv2", dict(n_boot=1, n_inviter=2))]:
        S = Solver(DIMS, **params(**kw))
        S.set_gauge(U)
        ed, fi = S.pack(eta), S.pack(init)
        step(torch, S, ed, fi)                       # warm
        ts, tv, info = step(torch, S, ed, fi)
        rows[name] = dict(t_setup=ts, t_solve=tv, n_gcr=info.n_gcr, n_little=info.n_little,
                          n_little_solves=info.n_little_solves, rel_residual=info.rel_residual)
        S.close()
        del ed, fi
        torch.cuda.empty_cache()
        log(f"{name}: setup {ts:.3f} s, {info.n_gcr} iterations, solve {tv:.3f} s")
    return rows


def mixed_precision_32x16(torch):
    """32 x 16^3, eps 0.4 (seed 3001), m0 = -0.3, Gaussian source (seed 3002):
    BF16 two-row links, FP32 Schwarz and inner little solves, FP64 GCR and
    projector; Schwarz block 4^4 or 8 x 4^3, then the little solver's grid,
    chosen by the autotuner on setup + solve time. Time to solution against the all-FP64 deflated solver
    and plain FP64 GCR on the same field. Errors: dirac_apply and one Schwarz
    application against the FP64 oracle; the solution against the all-FP64
    solve to 1e-12, and its true residual recomputed by the oracle's D."""
    import latgen
    import oracle
    from paper_0706_2298_amd import BF16, F32, F64, SOLVER_GCR, Solver, autotune, binding
    dims, m0 = (32, 16, 16, 16), -0.3
    U = latgen.make_links(dims, 0.4, 3001)
    eta = latgen.make_source(dims, 3002)
    init = latgen.make_init_fields(dims, 20, 3003)
    base = params(Ns=20, m0=m0, m0_setup=m0, link_prec=BF16, sap_prec=F32, little_prec=F32)
    base.pop("sap_block")
    cands = [dict(sap_block=sb, nmr=NMR, graph=False) for sb in [(4, 4, 4, 4), (8, 4, 4, 4)]]
    tuned = autotune.tune(dims, U, eta[None], init=init, params=base, cands=cands, cache=None, solves_per_setup=1,
                          reps=1)
    S = Solver(dims, sap_block=tuned["sap_block"], little_grid=tuned["little_grid"], **base)
    S.set_gauge(U)
    ed, initd = S.pack(eta), S.pack(init)
    S.setup(initd)
    S.solve(ed)
    _, t_setup = timed(torch, lambda: S.setup(initd))
    (psi, info), t_solve = timed(torch, lambda: S.solve(ed))
    psi = S.unpack(psi)[0]
    x = S.pack(eta, prec=F32)
    y = S.field(1, F32)
    binding.dirac_apply(S.ctx, x, y, 1, F32)
    dref = oracle.dirac(U, eta, m0, dims)
    d_err = float(np.linalg.norm(S.unpack(y, prec=F32)[0] - dref) / np.linalg.norm(dref))
    sap_gpu = S.unpack(S.sap(ed))[0]
    sap_ref = oracle.sap(U, eta, m0, dims, tuple(tuned["sap_block"]), NCY, NMR)
    s_err = float(np.linalg.norm(sap_gpu - sap_ref) / np.linalg.norm(sap_ref))
    S.close()
    out = dict(lattice=list(dims), m0=m0, autotune=dict(sap_block=list(tuned["sap_block"]), little_grid=tuned["little_grid"],
                                                         seconds=tuned["seconds"]),
               mixed=dict(t_setup=t_setup, t_solve=t_solve, n_gcr=info.n_gcr, n_little=info.n_little))
    # all-FP64 deflated solver on the same field and block shape (to 1e-10 for the
    # time, to 1e-12 for the reference solution)
    R = Solver(dims, **params(Ns=20, m0=m0, m0_setup=m0, sap_prec=F64, link_prec=F64, little_prec=F64,
                              sap_block=tuned["sap_block"]))
    R.set_gauge(U)
    ed, initd = R.pack(eta), R.pack(init)
    R.setup(initd)
    R.solve(ed)
    _, t_setup64 = timed(torch, lambda: R.setup(initd))
    (_, info64), t_solve64 = timed(torch, lambda: R.solve(ed))
    out["all_f64_dfl"] = dict(t_setup=t_setup64, t_solve=t_solve64, n_gcr=info64.n_gcr)
    R.close()
    R = Solver(dims, **params(Ns=20, m0=m0, m0_setup=m0, sap_prec=F64, link_prec=F64, little_prec=F64, tol=1e-12,
                              sap_block=tuned["sap_block"]))
    R.set_gauge(U)
    R.setup(R.pack(init))
    ref, _ = R.solve(R.pack(eta))
    ref = R.unpack(ref)[0]
    R.close()
    G = Solver(dims, **params(Ns=1, m0=m0, solver=SOLVER_GCR, nkv=32, maxiter=20000, sap_prec=F64, link_prec=F64))
    G.set_gauge(U)
    ed = G.pack(eta)
    (_, infog), t_gcr = timed(torch, lambda: G.solve(ed))
    out["gcr_f64"] = dict(t_solve=t_gcr, n_gcr=infog.n_gcr)
    G.close()
    del ed
    torch.cuda.empty_cache()
    res = float(np.linalg.norm(eta - oracle.dirac(U, psi, m0, dims)) / np.linalg.norm(eta))
    out.update(rel_residual_oracle_D=res, err_solution_vs_fp64_solve=float(np.linalg.norm(psi - ref) /
                                                                           np.linalg.norm(ref)),
               err_dirac_bf16_links_vs_oracle=d_err, err_sap_fp32_bf16_vs_oracle=s_err,
               speedup_vs_gcr_f64=t_gcr / (t_setup + t_solve))
    return out


def multi_rhs(torch):
    """12 point sources (x = 0, spin-colour 0..11) on 48 x 24^3 (seed 4001) and
    6 (spin-colour 0..5) on 32 x 16^3 (seed 4002), eps 0.4, m0 = -0.3, Ns = 24:
    one batched solve per lattice with graph replay against one-by-one solves
    on the same subspace and plain FP64 GCR (batched); plus dirac_apply on the
    12 sources in one launch."""
    import latgen
    from paper_0706_2298_amd import F64, SOLVER_GCR, Solver, binding
    out = {}
    for dims, seed, n in [((48, 24, 24, 24), 4001, 12), ((32, 16, 16, 16), 4002, 6)]:
        key = "x".join(map(str, dims))
        U = latgen.make_links(dims, 0.4, seed)
        src = latgen.point_sources(dims, range(n))
        init = latgen.make_init_fields(dims, 24, seed + 200)
        S = Solver(dims, **params(Ns=24, m0=-0.3, m0_setup=-0.3, nrhs_max=n))
        S.set_gauge(U)
        ed = S.pack(src)
        _, t_setup = timed(torch, lambda: S.setup(S.pack(init)))
        row = dict(nrhs=n, t_setup=t_setup)
        S.use_graphs(True)
        S.solve(ed)  # captures the step graphs
        (psi, infos), row["t_batched_graph"] = timed(torch, lambda: S.solve(ed))
        row["n_gcr_batched"] = [i.n_gcr for i in infos]
        row["max_rel_residual"] = max(i.rel_residual for i in infos)
        S.use_graphs(False)
        _, row["t_batched_direct"] = timed(torch, lambda: S.solve(ed))
        singles = []
        t_single = 0.0
        for j in range(n):
            ej = S.pack(src[j])
            (_, inf1), dt = timed(torch, lambda: S.solve(ej))
            t_single += dt
            singles.append(inf1.n_gcr)
        row["t_one_by_one"] = t_single
        row["n_gcr_single"] = singles
        row["speedup_batched_graph"] = t_single / row["t_batched_graph"]
        if n == 12:
            y = S.field(n, F64)
            t = time_events(torch, lambda: binding.dirac_apply(S.ctx, ed, y, n, F64), 10)
            vol = int(np.prod(dims))
            byts = (2 * 192 * n + 384) * vol  # spinors in and out per source, two-row links once
            row["dirac_nrhs12"] = dict(us=t * 1e6, gflops=FLOPS_PER_SITE * vol * n / t / 1e9,
                                       gbs=byts / t / 1e9, frac_hbm=byts / t / 1e9 / HBM_PEAK_GBS,
                                       bytes_per_site_per_rhs=byts / vol / n)
            del y
        S.close()
        del ed
        torch.cuda.empty_cache()
        G = Solver(dims, **params(Ns=1, m0=-0.3, solver=SOLVER_GCR, nkv=16, maxiter=20000, nrhs_max=n,
                                  sap_prec=F64, link_prec=F64))
        G.set_gauge(U)
        ed = G.pack(src)
        (_, infg), row["t_gcr_f64_batched"] = timed(torch, lambda: G.solve(ed))
        row["n_gcr_f64"] = [i.n_gcr for i in infg]
        G.close()
        del ed
        torch.cuda.empty_cache()
        row["speedup_vs_gcr_f64"] = row["t_gcr_f64_batched"] / (t_setup + row["t_batched_graph"])
        out[key] = row
        log(f"multi-rhs {key}: batched {row['t_batched_graph']:.3f} s, one by one {t_single:.3f} s, "
            f"plain GCR {row['t_gcr_f64_batched']:.3f} s")
    return out


def learned_subspace(torch, n_train=20, n_test=5, train_steps=300, m0=-0.56):
    """Start-field network: trained on 20 seeded 16^4 gauge fields (eps 0.5,
    seeds 5000..5019; targets = 24 inverse-iteration low modes, 3 steps, from
    seeded random fields), tested on 5 held-out 64 x 32^3 fields (seeds
    5100..5104) at m0 = -0.56: deflated SAP-GCR setup and solve times with the
    subspace grown from (a) random fields with 3 inverse-iteration steps,
    (b) network fields with 3 steps and (c) with 1 step, (d) network fields
    from the BF16-operand forward pass with 1 step and (e) with none, and
    plain FP64 GCR on the same field. The network is local (receptive field
    9^4) and the links are i.i.d. per site, so a 16^4 lattice has the local
    statistics of a 64 x 32^3 one."""
    import latgen
    from paper_0706_2298_amd import SOLVER_GCR, F64, Solver
    from paper_0706_2298_amd.learned import CHANNELS, StartFieldNet, make_targets
    tdims, eps, K = (16, 16, 16, 16), 0.5, 24
    prm = params(m0=m0, m0_setup=m0, n_inviter=0)
    S = Solver(tdims, **prm)
    links, targets = [], []
    t0 = time.perf_counter()
    for j in range(n_train):
        U = latgen.make_links(tdims, eps, 5000 + j)
        S.set_gauge(U)
        targets.append(make_targets(S, S.pack(latgen.make_init_fields(tdims, K, 5300 + j)), 3))
        links.append(U)
    t_targets = time.perf_counter() - t0
    net = StartFieldNet(S, latgen.net_init(CHANNELS, 5500))
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(train_steps):
        j = i % n_train
        S.set_gauge(links[j])
        losses.append(net.train_step(latgen.net_noise(tdims, 8000 + i), targets[j], K, lr=3e-3))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    weights = net.weights_numpy()
    S.close()
    del targets, net
    torch.cuda.empty_cache()
    T = Solver(DIMS, **prm)
    net = StartFieldNet(T, weights)
    # the BF16 forward keeps a BF16 copy of the weights, allocated on first use
    T.set_gauge(latgen.make_links(DIMS, eps, 5100))
    net.forward(torch.zeros(V * 24, dtype=torch.float32, device="cuda"), bf16=True)
    torch.cuda.synchronize()
    variants = [("random_k3", 3, None), ("learned_k3", 3, False), ("learned_k1", 1, False),
                ("learned_bf16_k1", 1, True), ("learned_bf16_k0", 0, True)]
    G = Solver(DIMS, **params(Ns=1, m0=m0, solver=SOLVER_GCR, nkv=32, maxiter=20000, sap_prec=F64, link_prec=F64))
    rows = []
    for j in range(n_test):
        seed = 5100 + j
        U = latgen.make_links(DIMS, eps, seed)
        eta = latgen.make_source(DIMS, seed + 100)
        T.set_gauge(U)
        ed = T.pack(eta)
        row = dict(seed=seed)
        noise = torch.tensor(latgen.net_noise(DIMS, seed + 400), dtype=torch.float32, device="cuda")
        for name, steps, bf16 in variants:
            # the random numbers of either start are generated and uploaded
            # before the clock starts
            if bf16 is None:
                f = T.pack(latgen.make_init_fields(DIMS, K, seed + 200))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            else:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                f = net.forward(noise, bf16=bf16)
            make_targets(T, f, steps)
            T.setup(f)
            torch.cuda.synchronize()
            t_setup = time.perf_counter() - t0
            (_, info), t_solve = timed(torch, lambda: T.solve(ed))
            row[name] = dict(n_gcr=info.n_gcr, t_setup=t_setup, t_solve=t_solve, status=info.status,
                             rel_residual=info.rel_residual, n_little=info.n_little)
            del f
        G.set_gauge(U)
        eg = G.pack(eta)
        (_, infog), t_g = timed(torch, lambda: G.solve(eg))
        row["gcr_f64"] = dict(n_gcr=infog.n_gcr, t_solve=t_g)
        del noise, eg, ed
        rows.append(row)
        log(f"learned: field {seed}: " + ", ".join(f"{k} {row[k]['n_gcr']} it" for k in row if k != "seed"))
    T.close()
    G.close()
    torch.cuda.empty_cache()
    mean = lambda k, q: float(np.mean([r[k][q] for r in rows]))
    summary = {k: dict(n_gcr=mean(k, "n_gcr"), t_setup=mean(k, "t_setup"), t_solve=mean(k, "t_solve"))
               for k, _, _ in variants}
    summary["gcr_f64"] = dict(n_gcr=mean("gcr_f64", "n_gcr"), t_solve=mean("gcr_f64", "t_solve"))
    return dict(train_lattice=list(tdims), test_lattice=list(DIMS), eps=eps, m0=m0, channels=list(CHANNELS),
                n_train_fields=n_train, train_steps=train_steps, t_targets=t_targets, t_train=t_train,
                loss_first10=float(np.mean(losses[:10])), loss_last10=float(np.mean(losses[-10:])), tests=rows,
                mean_over_tests=summary)


def workload_16x4(torch):
    """The 16^4 lattice at eps 0.4 and 0.6 (seeds 2001/2002), one setup
    (Ns = 20, 3 inverse-iteration steps) per field reused for m0 = -0.2, -0.3,
    -0.35: time per step of six solves, and the undeflated solvers."""
    import latgen
    from paper_0706_2298_amd import SOLVER_GCR, SOLVER_SAP_GCR, F64, Solver
    ctx = []
    for eps, seed in C2_FIELDS:
        U = latgen.make_links(C2_DIMS, eps, seed)
        S = Solver(C2_DIMS, **params(Ns=20, m0=C2_MASSES[0], m0_setup=min(C2_MASSES), little_prec=F64))
        S.set_gauge(U)
        ctx.append(dict(S=S, U=U, eps=eps, eta_h=latgen.make_source(C2_DIMS, seed + 100),
                        eta=S.pack(latgen.make_source(C2_DIMS, seed + 100)),
                        init=S.pack(latgen.make_init_fields(C2_DIMS, 20, seed + 200))))
    stats = []

    def one(record):
        for c in ctx:
            c["S"].setup(c["init"])
            for m in C2_MASSES:
                c["S"].set_mass(m)
                (_, info), t = timed(torch, lambda: c["S"].solve(c["eta"]))
                if record:
                    stats.append(dict(eps=c["eps"], m0=m, n_gcr=info.n_gcr, t_solve=t))
    one(False)
    _, dt = timed(torch, lambda: one(True))
    rows = []
    for c in ctx:
        c["S"].close()
        for solver, name in [(SOLVER_SAP_GCR, "sap_gcr"), (SOLVER_GCR, "gcr_f64")]:
            S = Solver(C2_DIMS, **params(solver=solver, nkv=32, Ns=1, maxiter=20000))
            S.set_gauge(c["U"])
            ed = S.pack(c["eta_h"])
            for m in C2_MASSES:
                S.set_mass(m)
                (_, info), t = timed(torch, lambda: S.solve(ed))
                rows.append(dict(solver=name, eps=c["eps"], m0=m, n_gcr=info.n_gcr, t_solve=t))
            S.close()
    torch.cuda.empty_cache()
    return dict(lattice=list(C2_DIMS), ms_per_step=dt * 1e3, solves_per_s=6 / dt, dfl_sap_gcr=stats,
                undeflated=rows)


def _oracle_units(threads_note=""):
    """Oracle unit costs on the 16^4 field of eps 0.5 (one Dirac application,
    one Schwarz application with 5 cycles, block Gram-Schmidt plus little
    operator for 24 fields, one little-operator application, one restriction
    plus prolongation with 24 fields)."""
    import latgen
    import oracle
    dims = (16, 16, 16, 16)
    U = latgen.make_links(dims, EPS, 6001)
    eta = latgen.make_source(dims, 6002)
    init = latgen.make_init_fields(dims, NS, 6003)
    t = {}
    t0 = time.perf_counter()
    oracle.dirac(U, eta, M0, dims)
    t["dirac"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.sap(U, eta, M0, dims, BLOCK, NCY, NMR)
    t["sap"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    Phi = oracle.block_gram_schmidt(init, dims, BLOCK)
    A = oracle.little_operator(U, Phi, M0, dims, BLOCK)
    t["subspace"] = time.perf_counter() - t0
    v = oracle.restrict(Phi, eta, dims, BLOCK)
    t0 = time.perf_counter()
    oracle.little_apply(A, v, dims, BLOCK)
    t["little_apply"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.prolong(Phi, oracle.restrict(Phi, eta, dims, BLOCK), dims, BLOCK)
    t["project"] = time.perf_counter() - t0
    t["threads"] = oracle.num_threads()
    return t


def cpu_baseline(prof, info):
    """The FP64 oracle on a bounded sample, scaled to the headline step.

    Sample: unit costs of the oracle on a 16^4 lattice (1/32 of the headline
    volume; every unit is linear in the volume): one Dirac application, one
    Schwarz application, the subspace build for 24 fields, one little-operator
    application and one restriction plus prolongation. The step's cost is the
    GPU step's own operation counts times these units times 32: setup (3
    inverse-iteration Schwarz applications per field, the subspace build) and
    solve (per GCR iteration one Schwarz application, two Dirac applications
    and two projections; per little GCR iteration two little-operator
    applications). Also the units with one thread (a subprocess with
    OMP_NUM_THREADS=1)."""
    units = _oracle_units()
    scale = V / 16 ** 4
    n_it = info.n_gcr + info.n_restarts
    n_little = prof["little_iterations"]
    est_setup = scale * (NINV * NS * units["sap"] + units["subspace"])
    est_solve = scale * (info.n_gcr * units["sap"] + 2 * n_it * units["dirac"] + 2 * n_it * units["project"]
                         + 2 * n_little * units["little_apply"])
    est = est_setup + est_solve
    one = None
    try:
        env = dict(os.environ, OMP_NUM_THREADS="1")
        code = ("import json, bench; print(json.dumps(bench._oracle_units()))")
        r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                           timeout=300)
        if r.returncode == 0:
            one = json.loads(r.stdout.strip().splitlines()[-1])
    except (subprocess.TimeoutExpired, ValueError, IndexError):
        one = None
    return dict(value=1.0 / est, unit="steps/s", cores=units["threads"], kind="oracle",
                sample=(f"oracle unit costs on 16^4 (eps 0.5): Dirac {units['dirac']:.3f}s, Schwarz application "
                        f"{units['sap']:.2f}s, 24-field subspace {units['subspace']:.2f}s, little apply "
                        f"{units['little_apply']:.4f}s, restrict+prolong {units['project']:.3f}s; x{scale:.0f} "
                        f"volume, times the GPU step's counts ({NINV}x{NS} setup Schwarz applications, "
                        f"{info.n_gcr} GCR iterations, {n_little} little iterations) -> {est_setup:.0f}s setup + "
                        f"{est_solve:.0f}s solve per step"),
                est_setup_s=est_setup, est_solve_s=est_solve, units=units, units_one_thread=one)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dirac", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the 32x16^3, multi-source and 16^4 runs")
    ap.add_argument("--no-learned", action="store_true", help="skip the start-field network training and tests")
    ap.add_argument("--learned-tests", type=int, default=5, help="held-out 64x32^3 fields for the network")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device copy (y = 1.0 * x), to scale HBM byte counters")
    ap.add_argument("--dirac-only", action="store_true", help="only the dirac_apply rates on 64x32^3")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; --gpus must be 1 (sharding over several GPUs "
                                   "is a design note, not built)"}))
        sys.exit(2)

    import torch
    from paper_0706_2298_amd import Solver
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(3)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        x = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_read_bytes": x.numel() * 8, "copy_write_bytes": y.numel() * 8, "dispatches": 5}))
        return

    if args.dirac_only:
        print(json.dumps(dirac_rates(torch)), flush=True)
        return

    log("generating inputs")
    U, eta_h, init_h = headline_inputs()
    S = Solver(DIMS, **params())
    S.set_gauge(U)
    eta, init = S.pack(eta_h), S.pack(init_h)
    torch.cuda.synchronize()

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step(torch, S, eta, init)
    log(f"timing {args.steps} steps")
    per = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        per.append(step(torch, S, eta, init))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    info = per[0][2]
    log(f"step {dt * 1e3:.1f} ms (setup {np.median([p[0] for p in per]) * 1e3:.1f} ms, "
        f"solve {np.median([p[1] for p in per]) * 1e3:.1f} ms, {info.n_gcr} iterations)")

    result = {
        "metric": "dirac_apply GFLOP/s + HBM GB/s; time-to-solution @ rel. residual 1e-10",
        "value": 1.0 / dt,
        "unit": "solves/s (one subspace setup + one solve each)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32 (FP64 GCR, projector and residual; FP32 Schwarz and inner little solves)",
        "data": "synthetic",
        "config": {"workload": "64x32^3 DFL+SAP+GCR, eps 0.5 (seed 5100), m0 -0.56: one setup (Ns 24, 3 "
                               "inverse-iteration steps, 4^4 blocks) + one solve to 1e-10 per step",
                   "lattice": list(DIMS), "Ns": NS, "n_inviter": NINV, "ncy": NCY, "nmr": NMR, "nkv": NKV,
                   "blocks": list(BLOCK)},
        "time_to_solution_s": {"setup": float(np.median([p[0] for p in per])),
                               "solve": float(np.median([p[1] for p in per])), "total": dt},
        "solve": dict(info.as_dict()),
    }
    if not args.no_profile:
        log("profiled step")
        prof = profiled(S, lambda: step(torch, S, eta, init))
        result["roofline"] = roofline(prof)
        result["kernel_time_per_step"] = {k: dict(seconds=prof[k][0], launches=prof[k][1])
                                          for k in prof if k != "little_iterations"}
        result["kernel_time_per_step"]["little_iterations"] = prof["little_iterations"]
    else:
        prof = None
    S.close()
    del eta, init
    torch.cuda.empty_cache()

    if not args.no_dirac:
        log("dirac_apply on 64x32^3")
        result["dirac_apply"] = dirac_rates(torch)
    if not args.no_compare:
        log("comparisons on the headline field")
        result["comparisons"] = comparisons(torch, U, eta_h, init_h)
    if not args.no_extras:
        log("mixed precision on 32x16^3")
        result["mixed_precision_32x16^3"] = mixed_precision_32x16(torch)
        log("multi-source batches")
        result["multi_rhs"] = multi_rhs(torch)
        log("16^4 workload")
        result["workload_16^4"] = workload_16x4(torch)
    if not args.no_learned:
        log("learned start fields")
        result["learned_subspace"] = learned_subspace(torch, n_test=args.learned_tests)
    if not args.no_cpu_baseline and prof is not None:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(prof, info)
    result["host"] = {"cpu": platform.processor() or platform.machine(), "nproc": os.cpu_count()}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
