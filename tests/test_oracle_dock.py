"""Pins for the oracle's Lamarckian GA and ADADELTA local search (CPU only).

The search is stochastic, so these pin its invariants and distributions:
exact evaluation accounting, elitism, uniform initial orientations
(Shoemake), the rank distribution of binary tournaments, crossover and
mutation structure, distinct local-search picks, ADADELTA convergence in a
bowl with a known minimum, and re-scoring of returned poses.
"""
import math

import numpy as np
import pytest

import oracle
import synth

T = synth.TYPE_ID


@pytest.fixture(scope="module")
def small(orc):
    rec = synth.receptor(17, 600, side=14.0)
    grid = synth.make_grid(24, 0.375, map_types=synth.SIX_TYPES)
    G = orc.grid(grid, rec)
    lig = synth.ligand(18, 16, 3)
    return grid, G, orc.ligand(lig)


def test_evaluation_accounting(orc, small):
    grid, G, L = small
    p = oracle.make_params(nrun=2, pop=12, max_gens=1000, max_evals=5000, ls_rate=0.2, ls_iters=20)
    n_ls = orc.n_ls(p)
    assert n_ls == 2
    per_gen = (12 - 1) + n_ls * 20
    geno, E, ev, gens = orc.dock(L, G, p, 5, 0)
    G_expect = (5000 - 12) // per_gen
    assert list(gens) == [G_expect] * 2
    assert list(ev) == [12 + G_expect * per_gen] * 2
    assert np.all(ev <= 5000)
    # generation cap binds first
    p2 = oracle.make_params(nrun=1, pop=12, max_gens=3, max_evals=10**9, ls_rate=0.2, ls_iters=20)
    _, _, ev2, gens2 = orc.dock(L, G, p2, 5, 0)
    assert gens2[0] == 3 and ev2[0] == 12 + 3 * per_gen


def test_elitism_and_rescoring(orc, small):
    grid, G, L = small
    best = []
    for gens in (0, 1, 3, 6, 10):
        p = oracle.make_params(nrun=1, pop=20, max_gens=gens, ls_rate=0.1, ls_iters=15)
        geno, E, _, _ = orc.dock(L, G, p, 99, 3)
        best.append(E[0])
        # the returned genotype re-scores to the returned energy
        assert orc.score(L, G, geno[0])[0] == pytest.approx(E[0], rel=1e-12, abs=1e-12)
    assert all(b2 <= b1 for b1, b2 in zip(best, best[1:]))
    assert best[-1] < best[0]


def test_docking_is_deterministic_and_thread_independent(orc, small):
    grid, G, L = small
    p = oracle.make_params(nrun=4, pop=10, max_gens=3, ls_rate=0.2, ls_iters=10)
    a = orc.dock(L, G, p, 7, 1, threads=1)
    b = orc.dock(L, G, p, 7, 1, threads=4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    c = orc.dock(L, G, p, 8, 1, threads=4)
    assert not np.array_equal(a[1], c[1])


def test_initial_population_is_uniform(orc, small):
    grid, G, L = small
    lo = np.array(grid.origin)
    hi = lo + np.array(grid.extent)
    q = []
    for i in range(3000):
        g = orc.init_individual(L, G, 12345, 2, 1, i)
        assert np.all(g[0:3] >= lo) and np.all(g[0:3] < hi)
        assert np.all(g[7:7 + L.n_tor] >= -math.pi) and np.all(g[7:7 + L.n_tor] < math.pi)
        assert np.all(g[7 + L.n_tor:] == 0)
        q.append(g[3:7])
    q = np.array(q)
    assert np.allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-14)
    # uniform on the 3-sphere: E[x_i^2] = 1/4 and E|x_i| = 4 / (3 pi) for every component
    assert np.allclose((q ** 2).mean(axis=0), 0.25, atol=0.02)
    assert np.allclose(np.abs(q).mean(axis=0), 4 / (3 * math.pi), atol=0.02)


def test_tournament_rank_distribution(orc, small):
    """tour_p = 1, no crossover or mutation: each child copies the better of two
    uniform picks, so P(rank r) = (2 (pop - r) - 1) / pop^2 (rank 0 = best)."""
    grid, G, L = small
    pop = 16
    p = oracle.make_params(pop=pop, cx_rate=0.0, mut_rate=0.0, tour_p=1.0)
    rng = np.random.default_rng(1)
    counts = np.zeros(pop)
    for gen in range(1, 400):
        old = rng.normal(size=(pop, 40))
        E = rng.permutation(pop).astype(np.float64)     # energy = rank
        new, newE = orc.ga_offspring(L, p, 77, 0, 0, gen, old, E)
        assert np.array_equal(new[0], old[int(np.argmin(E))]) and newE[0] == E.min()
        for i in range(1, pop):
            j = [k for k in range(pop) if np.array_equal(new[i], old[k])]
            assert len(j) == 1
            counts[int(E[j[0]])] += 1
    expect = np.array([(2 * (pop - r) - 1) / pop ** 2 for r in range(pop)])
    freq = counts / counts.sum()
    assert np.abs(freq - expect).max() < 0.012


def test_crossover_takes_contiguous_blocks(orc):
    lig = synth.ligand(3, 20, 6)
    L = orc.ligand(lig)
    pop, T_ = 12, L.n_tor
    p = oracle.make_params(pop=pop, cx_rate=1.0, mut_rate=0.0, tour_p=0.6)
    rng = np.random.default_rng(2)
    old = rng.normal(size=(pop, 40))
    E = rng.normal(size=pop)
    new, _ = orc.ga_offspring(L, p, 5, 0, 0, 1, old, E)
    blocks = [slice(0, 3), slice(3, 7)] + [slice(7 + k, 8 + k) for k in range(T_)]
    for i in range(1, pop):
        src = []
        for b in blocks:
            s = [k for k in range(pop) if np.array_equal(new[i][b], old[k][b])]
            assert len(s) == 1
            src.append(s[0])
        # at most two parents and the second parent's blocks form one contiguous range
        parents = sorted(set(src))
        assert len(parents) <= 2
        if len(parents) == 2:
            for par in parents:
                idx = [k for k, s in enumerate(src) if s == par]
                if idx[0] != 0 and idx[-1] != len(src) - 1:
                    assert idx == list(range(idx[0], idx[-1] + 1))


def test_mutation_bounds(orc):
    lig = synth.ligand(4, 20, 6)
    L = orc.ligand(lig)
    pop = 40
    p = oracle.make_params(pop=pop, cx_rate=0.0, mut_rate=1.0, tour_p=1.0)
    rng = np.random.default_rng(3)
    old = np.zeros((pop, 40))
    old[:, 0:3] = rng.normal(size=(pop, 3))
    old[:, 0] += 10.0 * np.arange(pop)           # parents 10 A apart: identifiable after mutation
    q = rng.normal(size=(pop, 4))
    old[:, 3:7] = q / np.linalg.norm(q, axis=1, keepdims=True)
    old[:, 7:7 + L.n_tor] = rng.uniform(-math.pi, math.pi, size=(pop, L.n_tor))
    E = np.arange(pop, dtype=np.float64)
    new, _ = orc.ga_offspring(L, p, 6, 0, 0, 1, old, E)
    angles = []
    for i in range(1, pop):
        a = [k for k in range(pop)]
        par = old[np.argmin([np.abs(new[i][0:3] - old[k][0:3]).max() for k in a])]
        d = new[i][0:3] - par[0:3]
        assert np.all(np.abs(d) <= p.mut_t) and np.all(d != 0)
        dth = (new[i][7:7 + L.n_tor] - par[7:7 + L.n_tor] + math.pi) % (2 * math.pi) - math.pi
        assert np.all(np.abs(dth) <= p.mut_theta + 1e-12)
        assert np.all(new[i][7:7 + L.n_tor] >= -math.pi) and np.all(new[i][7:7 + L.n_tor] < math.pi)
        cosang = abs(float(np.dot(new[i][3:7], par[3:7])))
        angles.append(2 * math.acos(min(1.0, cosang)))
        assert np.linalg.norm(new[i][3:7]) == pytest.approx(1.0, abs=1e-14)
    assert max(angles) <= p.mut_rot + 1e-9 and max(angles) > 0.3


def test_ls_pick_distinct_non_elite(orc):
    for gen in range(1, 50):
        pk = orc.ls_pick(11, 2, 3, gen, 150, 9)
        assert len(set(pk.tolist())) == 9 and pk.min() >= 1 and pk.max() <= 149
    allp = np.concatenate([orc.ls_pick(1, 0, 0, g, 10, 9) for g in range(1, 3)])
    assert sorted(allp[:9].tolist()) == list(range(1, 10))


def test_adadelta_descends_into_a_bowl(orc):
    """One atom in a map sampled from |p - p0|^2 (p0 a node): trilinear
    interpolation has its minimum exactly at p0, and ADADELTA gets there."""
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
    L = orc.ligand(lig)
    p = oracle.make_params()
    g = np.zeros(40)
    g[0:3] = p0 + np.array([1.8, -1.3, 0.9])
    g[3:7] = [0.5, 0.5, 0.5, 0.5]
    E0 = orc.score(L, G, g)[0]
    best, Eb = orc.adadelta(L, G, p, g, 300)
    assert E0 > 5.0
    # the interpolant is piecewise linear along each axis near p0 (a kink at the node), so
    # ADADELTA ends in a small oscillation around it rather than on it
    assert Eb < 0.1 and np.linalg.norm(best[0:3] - p0) < 0.15
    assert orc.score(L, G, best)[0] == pytest.approx(Eb, rel=1e-12, abs=1e-14)


def test_local_search_improves_random_poses(orc, small):
    grid, G, L = small
    p = oracle.make_params()
    for g in synth.random_genotypes(4, 5, L.n_tor, grid, margin=3.0, normalize_q=True):
        g = g.astype(np.float64)
        E0 = orc.score(L, G, g)[0]
        best, Eb = orc.adadelta(L, G, p, g, 100)
        assert Eb <= E0
        assert np.linalg.norm(best[3:7]) == pytest.approx(1.0, abs=1e-12)
