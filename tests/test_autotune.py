"""Autotuner selection and cache logic on the host (the measurement is replaced
by a fixed table), plus one GPU run on the 8^4 workload."""
import json

import numpy as np
import pytest

from paper_0706_2298_amd import autotune


def test_candidates_respect_block_constraints():
    c = autotune.candidates((8, 8, 8, 8))
    shapes = {x["sap_block"] for x in c}
    # 8 along any axis leaves one block there: only 4^4 is valid on 8^4
    assert shapes == {(4, 4, 4, 4)}
    c = autotune.candidates((32, 16, 16, 16))
    shapes = {x["sap_block"] for x in c}
    assert (8, 4, 4, 4) in shapes and (4, 4, 4, 4) in shapes
    assert len(c) == len(shapes) * len(autotune.NMR_CHOICES) * len(autotune.GRAPH_CHOICES)
    assert not autotune.valid_sap_block((16, 16, 16, 16), (8, 8, 4, 4))  # 1024 sites
    assert not autotune.valid_sap_block((24, 8, 8, 8), (8, 4, 4, 4))      # 3 blocks along x0


def test_tune_picks_fastest_and_caches(tmp_path):
    cache = str(tmp_path / "tune.json")
    dims = (32, 16, 16, 16)
    cands = autotune.candidates(dims)
    table = {i: 1.0 + 0.1 * i for i in range(len(cands))}
    table[3] = 0.5
    calls = []

    def measure(c):
        i = cands.index({k: c[k] for k in ("sap_block", "nmr", "graph")})
        calls.append(i)
        return table[i]

    eta = np.zeros((1, 4, 12))
    best = autotune.tune(dims, None, eta, params=dict(Ns=20), cands=cands, cache=cache, arch="gfx950",
                         measure=measure, little_grids=())
    assert best["cached"] is False and best["seconds"] == 0.5 and best["little_grid"] == 0
    assert (best["sap_block"], best["nmr"], best["graph"]) == (cands[3]["sap_block"], cands[3]["nmr"],
                                                             cands[3]["graph"])
    assert sorted(calls) == list(range(len(cands)))
    # second call: a cache hit, nothing measured
    calls.clear()
    again = autotune.tune(dims, None, eta, params=dict(Ns=20), cands=cands, cache=cache, arch="gfx950",
                          measure=measure)
    assert again["cached"] is True and calls == []
    assert again["sap_block"] == best["sap_block"]
    # another key (other Ns, other arch) is tuned separately
    autotune.tune(dims, None, eta, params=dict(Ns=24), cands=cands, cache=cache, arch="gfx950", measure=measure)
    autotune.tune(dims, None, eta, params=dict(Ns=20), cands=cands, cache=cache, arch="gfx942", measure=measure)
    assert len(json.load(open(cache))) == 3


def test_little_grid_candidates():
    # 32 x 16^3 with 4^4 deflation blocks: Nb = 512, default grid 128
    assert autotune.little_grid_candidates((32, 16, 16, 16)) == [0, 32, 64, 256]
    # 8^4: Nb = 16 blocks, default 4; every explicit choice exceeds Nb
    assert autotune.little_grid_candidates((8, 8, 8, 8)) == [0]
    # 64 x 32^3: Nb = 8192, default clamped to 256
    assert autotune.little_grid_candidates((64, 32, 32, 32)) == [0, 32, 64, 128]


def test_tune_second_stage_little_grid(tmp_path):
    cache = str(tmp_path / "tune.json")
    dims = (32, 16, 16, 16)
    cands = autotune.candidates(dims, nmr=(4,), graphs=(False,))
    seen = []

    def measure(c):
        seen.append(dict(c))
        t = 1.0 + 0.01 * cands.index({k: c[k] for k in ("sap_block", "nmr", "graph")})
        return t - (0.3 if c.get("little_grid") == 64 else 0.0)

    best = autotune.tune(dims, None, np.zeros((1, 4, 12)), params=dict(Ns=20), cands=cands, cache=cache,
                         arch="gfx950", measure=measure)
    # stage 1 at the default grid, stage 2 over the other grids for the winner (cands[0])
    assert [c.get("little_grid", 0) for c in seen[:len(cands)]] == [0] * len(cands)
    stage2 = seen[len(cands):]
    assert [c["little_grid"] for c in stage2] == [32, 64, 256]
    assert all(c["sap_block"] == cands[0]["sap_block"] for c in stage2)
    assert best["little_grid"] == 64 and abs(best["seconds"] - 0.7) < 1e-12
    hit = autotune.tune(dims, None, np.zeros((1, 4, 12)), params=dict(Ns=20), cands=cands, cache=cache,
                        arch="gfx950", measure=measure)
    assert hit["cached"] is True and hit["little_grid"] == 64


def test_tune_rejects_all_failed(tmp_path):
    with pytest.raises(RuntimeError):
        autotune.tune((16, 16, 16, 16), None, np.zeros((1, 4, 12)), cands=[dict(sap_block=(4, 4, 4, 4), nmr=4,
                      graph=False)], cache=None, arch="x", measure=lambda c: float("inf"))


@pytest.mark.gpu
def test_tune_on_gpu(tmp_path):
    import latgen
    print("[case] autotune 8^4", flush=True)
    dims = (8, 8, 8, 8)
    U = latgen.make_links(dims, 0.4, 1001)
    eta = latgen.make_source(dims, 1002)[None]
    init = latgen.make_init_fields(dims, 8, 1003)
    params = dict(Ns=8, m0=-0.2, m0_setup=-0.2, ncy=5, n_inviter=3, sap_prec=1, link_prec=1, little_prec=1)
    cands = autotune.candidates(dims, nmr=(3, 4))
    cache = str(tmp_path / "tune.json")
    best = autotune.tune(dims, U, eta, init=init, params=params, cands=cands, cache=cache, solves_per_setup=2,
                         reps=1)
    assert best["cached"] is False and np.isfinite(best["seconds"]) and best["little_grid"] == 0
    assert autotune.tune(dims, U, eta, init=init, params=params, cands=cands, cache=cache)["cached"] is True
