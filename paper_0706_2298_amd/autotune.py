"""Time-to-solution autotuner for the deflated SAP-GCR solver.

The Schwarz block shape and the number of minimal-residual steps change the
algorithm (section 6: the preconditioner, hence the iteration counts and the
inverse-iteration subspace), so candidates are ranked by measured wall time of
one subspace setup plus ``solves_per_setup`` solves on the caller's gauge
field, not by kernel time alone. Graph replay of the GCR steps is a third
axis. A second stage then tries, for the winner, the workgroup count of the
little solver (the grid of its one-launch GCR: more workgroups add apply
bandwidth and cost more per grid barrier, so the best count depends on the
block count and Ns). The winner is cached in a JSON file keyed by device
architecture and problem (lattice, deflation blocks, Ns, precisions, number of
sources), so a second call with the same key measures nothing.

Every measurement goes through the library's C ABI (Solver); nothing here
computes any part of the method.
"""
from __future__ import annotations

import itertools
import json
import os
import time
from typing import Callable, Iterable

import numpy as np

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_0706_2298_amd", "autotune.json")

# Schwarz block shapes tried (x0 first): the paper's 4^4 and 8x4^3 and the
# 8-long shapes along the other axes
SAP_SHAPES = [(4, 4, 4, 4), (8, 4, 4, 4), (4, 8, 4, 4), (4, 4, 8, 4), (4, 4, 4, 8)]
NMR_CHOICES = (3, 4, 5)
GRAPH_CHOICES = (False, True)
# workgroups of the little solver (0: the library's default, a quarter of the
# block count); the library clamps to the block count and to 256
LITTLE_GRID_CHOICES = (0, 32, 64, 128, 256)


def valid_sap_block(dims, sb) -> bool:
    """The library's constraints: even block count >= 2 per direction, <= 512 sites."""
    if int(np.prod(sb)) > 512:
        return False
    for L, b in zip(dims, sb):
        if L % b or (L // b) % 2 or L // b < 2:
            return False
    return True


def candidates(dims, shapes: Iterable = SAP_SHAPES, nmr: Iterable = NMR_CHOICES,
               graphs: Iterable = GRAPH_CHOICES) -> list[dict]:
    """All valid (sap_block, nmr, graph) combinations for the lattice."""
    out = []
    for sb, m, g in itertools.product(shapes, nmr, graphs):
        if valid_sap_block(dims, sb):
            out.append(dict(sap_block=tuple(sb), nmr=int(m), graph=bool(g)))
    return out


def little_grid_candidates(dims, dfl_block=(4, 4, 4, 4), choices: Iterable = LITTLE_GRID_CHOICES) -> list[int]:
    """Distinct effective little-solver grids for the lattice: 0 (the default,
    Nb / 4) first, then every explicit count below the block count Nb that
    differs from the default."""
    nb = int(np.prod([L // b for L, b in zip(dims, dfl_block)]))
    default = max(1, min(nb // 4, 256, nb))
    out = [0]
    for g in choices:
        g = int(g)
        if g > 0 and g <= nb and g != default and g not in out:
            out.append(g)
    return out


def cache_key(arch: str, dims, params: dict, nrhs: int) -> str:
    fields = [arch, "x".join(map(str, dims)), "b" + "x".join(map(str, params.get("dfl_block", (4, 4, 4, 4)))),
              f"Ns{params.get('Ns', 20)}", f"link{params.get('link_prec', 0)}", f"sap{params.get('sap_prec', 0)}",
              f"little{params.get('little_prec', 0)}", f"nrhs{nrhs}"]
    return "|".join(fields)


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def measure_solver(dims, U, eta, init, params: dict, cand: dict, solves_per_setup: int = 3,
                   reps: int = 2) -> float:
    """Seconds for one setup + solves_per_setup solves (best of reps), or inf on failure."""
    from . import Solver  # deferred: the GPU library is only needed to measure
    import torch

    kw = dict(params)
    kw["sap_block"] = cand["sap_block"]
    kw["nmr"] = cand["nmr"]
    kw["little_grid"] = int(cand.get("little_grid", kw.get("little_grid", 0)))
    nrhs = eta.shape[0] if eta.ndim == 3 else 1
    kw["nrhs_max"] = max(kw.get("nrhs_max", 1), nrhs)
    S = Solver(dims, **kw)
    try:
        S.set_gauge(U)
        if cand["graph"]:
            S.use_graphs(True)
        ed = S.pack(eta)
        init_d = S.pack(init) if init is not None else None
        best = float("inf")
        for _ in range(reps + 1):  # first round warms up (and captures graphs)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S.setup(init_d)
            ok = True
            for _ in range(solves_per_setup):
                _, info = S.solve(ed)
                infos = info if isinstance(info, list) else [info]
                ok &= all(i.status == 0 for i in infos)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if not ok:
                return float("inf")
            best = min(best, dt)
        return best
    finally:
        S.close()


def tune(dims, U, eta, init=None, params: dict | None = None, cands: list[dict] | None = None,
         cache: str | None = DEFAULT_CACHE, arch: str | None = None, solves_per_setup: int = 3, reps: int = 2,
         measure: Callable | None = None, verbose: bool = False, little_grids: Iterable | None = None) -> dict:
    """Pick the fastest candidate for this problem; returns {sap_block, nmr, graph, little_grid, seconds, cached}.

    Stage 1 ranks ``cands`` (Schwarz block, MR steps, graphs) at the default
    little-solver grid; stage 2 tries ``little_grids`` (default: every
    distinct grid of ``little_grid_candidates``) for the stage-1 winner.
    ``measure(cand) -> seconds`` replaces the GPU measurement when given
    (used by the host-side tests of the selection and cache logic).
    """
    params = dict(params or {})
    nrhs = eta.shape[0] if np.ndim(eta) == 3 else 1
    if arch is None:
        import torch
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = cache_key(arch, dims, params, nrhs)
    data = _load(cache) if cache else {}
    if key in data:
        hit = dict(data[key])
        hit["sap_block"] = tuple(hit["sap_block"])
        hit["cached"] = True
        return hit
    cands = cands if cands is not None else candidates(dims)
    if not cands:
        raise ValueError(f"no valid Schwarz block shape for lattice {dims}")
    if measure is None:
        measure = lambda c: measure_solver(dims, U, eta, init, params, c, solves_per_setup, reps)  # noqa: E731
    timings = []
    for c in cands:
        t = float(measure(c))
        timings.append((t, c))
        if verbose:
            print(f"[autotune] {c} -> {t * 1e3:.2f} ms", flush=True)
    t_best, best = min(timings, key=lambda tc: tc[0])
    if not np.isfinite(t_best):
        raise RuntimeError("autotune: no candidate converged")
    best = dict(best, little_grid=int(best.get("little_grid", params.get("little_grid", 0))))
    grids = list(little_grids) if little_grids is not None else little_grid_candidates(
        dims, params.get("dfl_block", (4, 4, 4, 4)))
    for lg in grids:
        if int(lg) == best["little_grid"]:
            continue
        c = dict(best, little_grid=int(lg))
        t = float(measure(c))
        if verbose:
            print(f"[autotune] {c} -> {t * 1e3:.2f} ms", flush=True)
        if t < t_best:
            t_best, best = t, c
    out = dict(sap_block=list(best["sap_block"]), nmr=best["nmr"], graph=best["graph"],
               little_grid=best["little_grid"], seconds=t_best)
    if cache:
        data = _load(cache)
        data[key] = out
        _store(cache, data)
    out = dict(out)
    out["sap_block"] = tuple(out["sap_block"])
    out["cached"] = False
    return out
