"""Pins for the oracle's Solis-Wets local search and the autostop rule
(CPU only).

Solis-Wets accepts only improvements, so at a strict minimum every
iteration fails twice and the step halves every sw_max_fail iterations: the
evaluation count is then a closed form.  Its deviates are standard normal
(moments over many draws), the search descends into a bowl with a known
minimum, never worsens the energy and respects its evaluation budget.
Autostop on a landscape where every pose has the same energy stops a run
after exactly ten recorded generations; a zero threshold never stops.
"""
import math

import numpy as np
import pytest

import oracle
import synth

T = synth.TYPE_ID


def bowl_setup(orc):
    grid = synth.make_grid(21, 0.375, map_types=[T["C"]])
    nx = 21
    z, y, x = np.meshgrid(np.arange(nx), np.arange(nx), np.arange(nx), indexing="ij")
    p0 = np.array(grid.origin) + 0.375 * np.array([12, 9, 10])
    P = [grid.origin[0] + 0.375 * x, grid.origin[1] + 0.375 * y, grid.origin[2] + 0.375 * z]
    bowl = (P[0] - p0[0]) ** 2 + (P[1] - p0[1]) ** 2 + (P[2] - p0[2]) ** 2
    vals = np.stack([bowl, np.zeros_like(bowl), np.zeros_like(bowl)]).astype(np.float32)
    G = orc.grid(grid, values=vals)
    lig = synth.Ligand(np.array([T["C"]], np.int32), np.zeros(1, np.float32), np.zeros((1, 3), np.float32),
                       np.zeros((0, 2), np.int32), np.zeros(0, np.uint8))
    return grid, G, orc.ligand(lig), p0


def test_deviates_are_standard_normal(orc):
    z = np.array([orc.sw_deviate(7, 1, 2, 3, 4, it, k) for it in range(2500) for k in range(8)])
    assert abs(z.mean()) < 0.03 and abs(z.var() - 1.0) < 0.05
    assert abs(np.mean(z ** 3)) < 0.1 and abs(np.mean(z ** 4) - 3.0) < 0.25
    # the two members of a Box-Muller pair are uncorrelated
    a = z.reshape(-1, 2)
    assert abs(np.corrcoef(a[:, 0], a[:, 1])[0, 1]) < 0.05
    assert orc.sw_deviate(7, 1, 2, 3, 4, 5, 6) == orc.sw_deviate(7, 1, 2, 3, 4, 5, 6)
    assert orc.sw_deviate(7, 1, 2, 3, 4, 5, 6) != orc.sw_deviate(8, 1, 2, 3, 4, 5, 6)


def test_at_a_strict_minimum_every_step_fails(orc):
    grid, G, L, p0 = bowl_setup(orc)
    g = np.zeros(40)
    g[0:3] = p0
    g[3:7] = [1, 0, 0, 0]
    E0 = orc.score(L, G, g)[0]
    assert E0 == pytest.approx(0.0, abs=1e-12)
    for rho0, lb, fails in [(1.0, 0.01, 4), (1.0, 0.01, 3), (0.5, 0.1, 2)]:
        p = oracle.make_params(sw_rho=rho0, sw_rho_lb=lb, sw_max_fail=fails)
        best, Eb, used = orc.solis_wets(L, G, p, g, 10**6, 3, 0, 0, 1, 1, E_in=E0)
        halvings = math.floor(math.log2(rho0 / lb)) + 1     # rho halves until it is below lb
        assert used == 2 * fails * halvings
        assert Eb == E0 and np.array_equal(best, g)


def test_descends_into_a_bowl_and_never_worsens(orc):
    grid, G, L, p0 = bowl_setup(orc)
    p = oracle.make_params()
    for s in range(5):
        g = np.zeros(40)
        g[0:3] = p0 + np.random.default_rng(s).uniform(-2, 2, 3)
        g[3:7] = [0.5, 0.5, 0.5, 0.5]
        E0 = orc.score(L, G, g)[0]
        best, Eb, used = orc.solis_wets(L, G, p, g, 300, 11, 0, 0, 1, s + 1)
        assert used <= 300
        assert Eb <= E0 and Eb < 0.05
        assert orc.score(L, G, best)[0] == pytest.approx(Eb, rel=1e-12, abs=1e-14)


def test_budget_and_degenerate_cases(orc):
    grid, G, L, p0 = bowl_setup(orc)
    g = np.zeros(40)
    g[0:3] = p0 + 1.0
    g[3:7] = [1, 0, 0, 0]
    E0 = orc.score(L, G, g)[0]
    p = oracle.make_params()
    for budget in (1, 2, 3, 17):
        _, Eb, used = orc.solis_wets(L, G, p, g, budget, 5, 0, 0, 1, 1, E_in=E0)
        assert used == budget and Eb <= E0
    # without a known start energy the start is evaluated first (one evaluation)
    _, Eb, used = orc.solis_wets(L, G, p, g, 1, 5, 0, 0, 1, 1)
    assert used == 1 and Eb == E0
    # a lower bound above the start step: no iteration
    p2 = oracle.make_params(sw_rho=0.1, sw_rho_lb=0.2)
    best, Eb, used = orc.solis_wets(L, G, p2, g, 300, 5, 0, 0, 1, 1, E_in=E0)
    assert used == 0 and Eb == E0 and np.array_equal(best, g)


def test_docking_with_solis_wets_accounts_evaluations(orc):
    rec = synth.receptor(17, 600, side=14.0)
    grid = synth.make_grid(24, 0.375, map_types=synth.SIX_TYPES)
    G = orc.grid(grid, rec)
    L = orc.ligand(synth.ligand(18, 16, 3))
    p = oracle.make_params(nrun=3, pop=12, max_gens=1000, max_evals=4000, ls_rate=0.2, ls_iters=40, ls_method=1)
    geno, E, ev, gens = orc.dock(L, G, p, 5, 0)
    n_ls = orc.n_ls(p)
    for r in range(3):
        ls_evals = ev[r] - 12 - gens[r] * 11
        assert 0 < ls_evals <= gens[r] * n_ls * 40
        assert ev[r] <= 4000 and ev[r] + 11 + n_ls * 40 > 4000 or gens[r] == 1000
        assert orc.score(L, G, geno[r])[0] == pytest.approx(E[r], rel=1e-12, abs=1e-12)
    # the same seed gives the same runs; ADADELTA differs
    geno2, E2, ev2, gens2 = orc.dock(L, G, p, 5, 0)
    assert np.array_equal(E, E2) and np.array_equal(ev, ev2)
    pa = oracle.make_params(nrun=3, pop=12, max_gens=1000, max_evals=4000, ls_rate=0.2, ls_iters=40)
    assert not np.array_equal(orc.dock(L, G, pa, 5, 0)[1], E)


def test_autostop_on_a_flat_landscape(orc):
    grid = synth.make_grid(12, 0.375, map_types=[T["C"]])
    vals = np.zeros((3, 12, 12, 12), np.float32)
    G = orc.grid(grid, values=vals)
    lig = synth.Ligand(np.array([T["C"]], np.int32), np.zeros(1, np.float32), np.zeros((1, 3), np.float32),
                       np.zeros((0, 2), np.int32), np.zeros(0, np.uint8))
    L = orc.ligand(lig)
    base = dict(nrun=2, pop=10, max_gens=50, max_evals=10**9, ls_rate=0.2, ls_iters=5)
    for method in (0, 1):
        # every energy is 0: ten recorded best energies (generations 0..9) have std 0
        _, _, ev, gens = orc.dock(L, G, oracle.make_params(**base, ls_method=method, autostop=1), 1, 0)
        assert list(gens) == [9, 9]
        # a zero threshold never stops a run
        _, _, _, gens0 = orc.dock(L, G, oracle.make_params(**base, ls_method=method, autostop=1, stop_std=0.0), 1, 0)
        assert list(gens0) == [50, 50]


def test_autostop_stops_a_converging_run_early(orc):
    rec = synth.receptor(17, 600, side=14.0)
    grid = synth.make_grid(24, 0.375, map_types=synth.SIX_TYPES)
    G = orc.grid(grid, rec)
    L = orc.ligand(synth.ligand(18, 16, 3))
    kw = dict(nrun=2, pop=30, max_gens=400, max_evals=10**9, ls_rate=0.1, ls_iters=30)
    g_off, E_off = orc.dock(L, G, oracle.make_params(**kw), 9, 0)[3], None
    _, E_on, _, g_on = orc.dock(L, G, oracle.make_params(**kw, autostop=1, stop_std=0.15), 9, 0)
    assert np.all(g_off == 400)
    assert np.all(g_on < 400) and np.all(g_on >= 9)
