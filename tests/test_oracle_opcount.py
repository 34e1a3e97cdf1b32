"""FLOP models of the evaluation, pinned by the op-counting build of the
oracle (oracle/opcount.hpp: oracle.c compiled unchanged as C++ with a double
that counts add, sub, mul, div and transcendentals, one each).

- The counted work of one energy + gradient evaluation decomposes exactly as
  54 + 227 N + 58 D + 27 T + sum over pairs of (28 + the pair functions'
  count at that pair's distance), N atoms, T torsions, D the (atom, torsion
  moving it) count; the pair functions cost 78, one more below the smoothing
  band and one more for an H-bond pair.
- bench.oracle_flops_per_eval (106 per pair) is a lower bound of that count
  and within one operation per pair of it.
- bench.flops_per_eval, the minimal count the roofline uses (constants
  hoisted), is below the oracle's count for every ligand.
"""
import importlib.util
import os

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SIZES = [(1, 0), (2, 0), (5, 1), (10, 2), (15, 3), (24, 5), (30, 8), (37, 9), (45, 12), (60, 15), (64, 16),
         (80, 20), (100, 32), (128, 32), (20, 0), (40, 20), (50, 30)]


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def oc(ff):
    return oracle.Oracle(ff, counting=True)


@pytest.fixture(scope="module")
def big_site(oc):
    # a 32.6 A box: every atom of every pose below stays inside (no restraint branch)
    rec = synth.receptor(11, 300, side=30.0)
    grid = synth.make_grid(88, 0.375, map_types=synth.ALL_TYPES)
    return grid, oc.grid(grid, rec)


def depth_sum(L):
    return sum(int(L.torsion(k)[3].sum()) for k in range(L.n_tor))


def test_counting_build_computes_the_same_values(ff, oc, orc, big_site):
    grid, Gc = big_site
    G = orc.grid(grid, values=Gc.values())
    lig = synth.ligand(7, 30, 6)
    Lc, L = oc.ligand(lig), orc.ligand(lig)
    g = np.zeros(40)
    g[:3] = grid.center
    g[3:7] = [0.6, 0.0, 0.8, 0.0]
    g[7:13] = [0.3, -1.0, 2.0, 0.1, -0.4, 1.5]
    E1, g1, t1 = oc.score(Lc, Gc, g)
    E2, g2, t2 = orc.score(L, G, g)
    assert E1 == E2 and np.array_equal(g1, g2) and np.array_equal(t1, t2)


def test_pair_function_counts(oc):
    # C-C: R = 4.0 A, band [3.75, 4.25]; OA-HD: H-bond, R_hb = 1.9 A, band [1.65, 2.15]
    C, OA, HD = synth.TYPE_ID["C"], synth.TYPE_ID["OA"], synth.TYPE_ID["HD"]
    count = lambda ti, tj, r: oc.opcount(oc.pair, ti, 0.1, tj, -0.2, r)[1]["total"]
    assert count(C, C, 5.0) == 78 and count(C, C, 4.0) == 78 and count(C, C, 3.0) == 79
    assert count(C, C, 0.001) == 79
    assert count(OA, HD, 5.0) == 79 and count(OA, HD, 1.9) == 79 and count(OA, HD, 1.0) == 80


def test_score_count_decomposes_exactly(oc, big_site):
    grid, G = big_site
    rng = np.random.default_rng(0)
    b = _bench()
    for s, (n, t) in enumerate(SIZES):
        lig = synth.ligand(500 + s, n, t)
        L = oc.ligand(lig)
        D = depth_sum(L)
        pairs = L.pairs()
        info = dict(n_pairs=L.n_pairs, n_atoms=L.n, n_torsions=L.n_tor, depth_sum=D)
        for rep in range(3):
            g = np.zeros(40)
            g[:3] = np.array(grid.center) + rng.normal(0, 1, 3)
            q = rng.normal(size=4)
            g[3:7] = q / np.linalg.norm(q)
            g[7:7 + L.n_tor] = rng.uniform(-np.pi, np.pi, L.n_tor) if rep else 0.0
            (_, c) = oc.opcount(oc.score, L, G, g)
            xyz = oc.pose(L, g)
            cp = sum(oc.opcount(oc.pair, int(lig.types[i]), 0.1, int(lig.types[j]), -0.1,
                                float(np.linalg.norm(xyz[i] - xyz[j])))[1]["total"] for i, j in pairs)
            assert c["total"] == 54 + 227 * L.n + 58 * D + 27 * L.n_tor + 28 * L.n_pairs + cp, (n, t, rep)
            model = b.oracle_flops_per_eval(info)
            assert model <= c["total"] <= model + 2 * L.n_pairs, (n, t, rep)


def test_minimal_model_is_below_the_oracle_count(oc):
    b = _bench()
    for s, (n, t) in enumerate(SIZES):
        L = oc.ligand(synth.ligand(500 + s, n, t))
        info = dict(n_pairs=L.n_pairs, n_atoms=L.n, n_torsions=L.n_tor, depth_sum=depth_sum(L))
        f_min, f_orc = b.flops_per_eval(info, True), b.oracle_flops_per_eval(info)
        assert 0.4 * f_orc <= f_min <= f_orc, (n, t, f_min, f_orc)
