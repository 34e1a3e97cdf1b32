"""GPU Solis-Wets local search and autostop against the oracle.

Exact where the method fixes the result: at a strict minimum every step
fails, so the evaluation count is a closed form and the pose is unchanged;
on a landscape where every pose scores the same, autostop ends every run
after exactly ten recorded generations.  Elsewhere the searches are
stochastic and compared like the ADADELTA search: most individual
trajectories follow the oracle's (the same random streams; FP32 genes and
deviates on the GPU), evaluation accounting holds, returned poses re-score,
results are reproducible, and best-energy distributions over independent
streams agree (Mann-Whitney).
"""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

T = synth.TYPE_ID


@pytest.fixture(scope="module")
def pkg():
    import torch
    assert torch.cuda.is_available()
    import paper_2007_03678_amd as pkg
    pkg.lib()
    return pkg


def one_atom():
    return synth.Ligand(np.array([T["C"]], np.int32), np.zeros(1, np.float32), np.zeros((1, 3), np.float32),
                        np.zeros((0, 2), np.int32), np.zeros(0, np.uint8))


def test_solis_wets_at_a_strict_minimum(pkg, ff, orc):
    grid = synth.make_grid(21, 0.375, map_types=[T["C"]])
    nx = 21
    z, y, x = np.meshgrid(np.arange(nx), np.arange(nx), np.arange(nx), indexing="ij")
    p0 = np.array(grid.origin) + 0.375 * np.array([12, 9, 10])
    P = [grid.origin[0] + 0.375 * x, grid.origin[1] + 0.375 * y, grid.origin[2] + 0.375 * z]
    bowl = (P[0] - p0[0]) ** 2 + (P[1] - p0[1]) ** 2 + (P[2] - p0[2]) ** 2
    vals = np.stack([bowl, np.zeros_like(bowl), np.zeros_like(bowl)]).astype(np.float32)
    ctx = pkg.create(ff, 0)
    ctx.ad_load_grids(grid, vals)
    batch = ctx.ad_load_ligands([one_atom()])
    g = np.zeros((3, 40), np.float32)
    g[:, 0:3] = p0
    g[:, 3:7] = [1, 0, 0, 0]
    for rho0, lb, fails in [(1.0, 0.01, 4), (1.0, 0.01, 3), (0.5, 0.1, 2)]:
        p = pkg.make_params(sw_rho=rho0, sw_rho_lb=lb, sw_max_fail=fails)
        best, E, used = ctx.ad_solis_wets(batch, np.zeros(3, np.int32), g, p, 10**6, 3)
        halvings = math.floor(math.log2(rho0 / lb)) + 1
        assert np.all(used == 1 + 2 * fails * halvings)
        assert np.all(E == 0.0) and np.array_equal(best, g)
    # away from the minimum it descends
    g2 = g.copy()
    g2[:, 0:3] += np.array([1.3, -0.9, 0.7], np.float32)
    best, E, used = ctx.ad_solis_wets(batch, np.zeros(3, np.int32), g2, pkg.make_params(), 300, 4)
    assert np.all(E < 0.05) and np.all(used <= 300)
    batch.free()
    ctx.close()


@pytest.fixture(scope="module")
def setup(pkg, ff, orc):
    rec = synth.receptor(31, 1200, side=16.0)
    grid = synth.make_grid(32, 0.375, map_types=synth.SIX_TYPES)
    G = orc.grid(grid, rec)
    ctx = pkg.create(ff, 0)
    ctx.ad_load_grids(grid, G.values())
    yield ctx, grid, G
    ctx.close()


def test_solis_wets_follows_the_oracle(pkg, setup, orc):
    ctx, grid, G = setup
    ligs = [synth.ligand(81, 14, 3), synth.ligand(82, 30, 8)]
    batch = ctx.ad_load_ligands(ligs)
    OL = [orc.ligand(l) for l in ligs]
    n = 40
    idx = np.array([i % 2 for i in range(n)], np.int32)
    nt = np.array([ligs[i].n_torsions for i in idx])
    g = synth.random_genotypes(5, n, nt, grid, margin=3.0, normalize_q=True)
    p = pkg.make_params()
    po = oracle.make_params()
    seed = (11 << 32) | 13
    best, E, used = ctx.ad_solis_wets(batch, idx, g, p, 30, seed)
    agree = 0
    for i in range(n):
        bo, Eo, uo = orc.solis_wets(OL[idx[i]], G, po, g[i].astype(np.float64), 30, seed, int(idx[i]), 0, 0, i)
        assert E[i] <= orc.score(OL[idx[i]], G, g[i].astype(np.float64))[0] + 1e-3   # never worse than the start
        Er = orc.score(OL[idx[i]], G, best[i].astype(np.float64))[0]
        assert abs(Er - E[i]) <= max(1e-3, 1e-5 * abs(Er))                          # returned pose re-scores
        if used[i] == uo and abs(E[i] - Eo) <= max(1e-3, 1e-4 * abs(Eo)):
            agree += 1
    assert agree >= 0.8 * n, agree
    batch.free()


def small_params(pkg, **kw):
    d = dict(nrun=4, pop=30, max_gens=1000, max_evals=6000, ls_rate=0.1, ls_iters=40, ls_method=1)
    d.update(kw)
    return pkg.make_params(**d)


def test_docking_with_solis_wets(pkg, setup, orc):
    ctx, grid, G = setup
    ligs = [synth.ligand(90 + i, n, t) for i, (n, t) in enumerate([(12, 2), (26, 6), (44, 12), (70, 20)])]
    batch = ctx.ad_load_ligands(ligs)
    OL = [orc.ligand(l) for l in ligs]
    p = small_params(pkg)
    r = ctx.ad_dock_batch(batch, p, 21, per_run=True)
    n_ls = 3
    for l in range(4):
        ev = int(r["evals"][l])
        assert ev <= 4 * 6000
        Eo, _, To = orc.score(OL[l], G, r["best_genotype"][l].astype(np.float64))
        assert abs(r["best_energy"][l] - Eo) <= max(1e-3, 1e-5 * abs(Eo))
        assert r["best_energy"][l] == r["run_energy"][l].min()
        Er, _, _ = ctx.ad_score_poses(batch, np.full(4, l, np.int32), r["run_genotype"][l])
        assert np.array_equal(Er, r["run_energy"][l])
    # the cap: no run could have afforded one more generation
    gens = r["generations"]
    assert np.all(gens >= 1)
    # reproducible; a subset docks the same
    r2 = ctx.ad_dock_batch(batch, p, 21, per_run=True)
    assert np.array_equal(r["run_energy"], r2["run_energy"]) and np.array_equal(r["evals"], r2["evals"])
    r3 = ctx.ad_dock_select(batch, np.array([3, 1], np.int32), p, 21, per_run=True)
    assert np.array_equal(r3["run_energy"], r["run_energy"][[3, 1]])
    # Solis-Wets differs from ADADELTA
    ra = ctx.ad_dock_batch(batch, small_params(pkg, ls_method=0), 21)
    assert not np.array_equal(ra["best_energy"], r["best_energy"])
    batch.free()


def test_autostop_on_a_flat_landscape(pkg, ff, orc):
    grid = synth.make_grid(12, 0.375, map_types=[T["C"]])
    ctx = pkg.create(ff, 0)
    ctx.ad_load_grids(grid, np.zeros((3, 12, 12, 12), np.float32))
    batch = ctx.ad_load_ligands([one_atom(), one_atom()])
    base = dict(nrun=3, pop=10, max_gens=50, max_evals=10**9, ls_rate=0.2, ls_iters=5)
    for method in (0, 1):
        r = ctx.ad_dock_batch(batch, pkg.make_params(**base, ls_method=method, autostop=1), 1)
        assert np.all(r["generations"] == 9)
        if method == 0:
            assert np.all(r["evals"] == 3 * (10 + 9 * (9 + 2 * 5)))
        r0 = ctx.ad_dock_batch(batch, pkg.make_params(**base, ls_method=method, autostop=1, stop_std=0.0), 1)
        assert np.all(r0["generations"] == 50)
    batch.free()
    ctx.close()


def test_autostop_ends_converged_runs_early(pkg, setup):
    ctx, grid, G = setup
    batch = ctx.ad_load_ligands([synth.ligand(95, 16, 3)] * 4)
    kw = dict(nrun=4, pop=30, max_gens=300, max_evals=10**9, ls_rate=0.1, ls_iters=30)
    off = ctx.ad_dock_batch(batch, pkg.make_params(**kw), 5, per_run=True)
    on = ctx.ad_dock_batch(batch, pkg.make_params(**kw, autostop=1), 5, per_run=True)
    assert np.all(off["generations"] == 300)
    assert np.all(on["generations"] < 300) and np.all(on["generations"] >= 9)
    assert np.all(on["evals"] < off["evals"])
    batch.free()


def test_solis_wets_docking_statistics_match_oracle(pkg, ff, orc):
    """24 independent streams of a 16-atom ligand (4 runs x pop 40, 30
    generations, Solis-Wets 60 evaluations on 10 %): GPU and oracle best
    energies are not distinguishable."""
    from scipy.stats import mannwhitneyu
    rec = synth.receptor(31, 1200, side=16.0)
    grid = synth.make_grid(32, 0.375, map_types=synth.SIX_TYPES)
    G = orc.grid(grid, rec)
    lig = synth.ligand(97, 16, 4)
    ctx = pkg.create(ff, 0)
    ctx.ad_load_grids(grid, G.values())
    n = 24
    batch = ctx.ad_load_ligands([lig] * n)
    kw = dict(nrun=4, pop=40, max_gens=30, ls_rate=0.1, ls_iters=60, ls_method=1)
    r = ctx.ad_dock_batch(batch, pkg.make_params(**kw), 8)
    L = orc.ligand(lig)
    eo = np.array([orc.dock(L, G, oracle.make_params(**kw), 8, k)[1].min() for k in range(n)])
    eg = r["best_energy"].astype(np.float64)
    pv = mannwhitneyu(eg, eo).pvalue
    assert pv > 0.01, (pv, np.sort(eg), np.sort(eo))
    assert abs(np.median(eg) - np.median(eo)) < 0.3 + 0.05 * abs(np.median(eo))
    batch.free()
    ctx.close()
