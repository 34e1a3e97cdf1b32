"""Checks of the seeded input generators (CPU): the ligands they emit are
valid typed trees with the stated geometry, for the Python and the C
generator alike."""
import numpy as np
import pytest

import synth


def check_ligand(lig, min_nonlocal=2.0):
    n = lig.n_atoms
    b = np.asarray(lig.bonds).reshape(-1, 2)
    assert len(b) == n - 1 and len(lig.rotatable) == n - 1
    # a tree: n-1 bonds connecting every atom
    parent = list(range(n))

    def find(u):
        while parent[u] != u:
            parent[u] = parent[parent[u]]
            u = parent[u]
        return u

    for u, v in b:
        ru, rv = find(int(u)), find(int(v))
        assert ru != rv
        parent[ru] = rv
    deg = np.bincount(b.ravel(), minlength=n) if n > 1 else np.zeros(1, int)
    for i in range(n):
        assert deg[i] <= synth.MAX_VALENCE[synth.TYPE_NAMES[lig.types[i]]]
        if synth.TYPE_NAMES[lig.types[i]] == "HD":
            assert deg[i] == 1
            j = int(b[np.where((b == i).any(axis=1))[0][0]].sum() - i)
            assert synth.TYPE_NAMES[lig.types[j]] in ("N", "OA")
    if n > 1:
        d = np.linalg.norm(lig.xyz[b[:, 0]] - lig.xyz[b[:, 1]], axis=1)
        assert d.min() >= 1.0 - 1e-5 and d.max() <= 1.55 + 1e-5
    # rotatable bonds join two atoms of degree >= 2
    for k in np.where(lig.rotatable)[0]:
        assert deg[b[k, 0]] >= 2 and deg[b[k, 1]] >= 2
    # bond-path distances and clash rules
    adj = [[] for _ in range(n)]
    for u, v in b:
        adj[u].append(v)
        adj[v].append(u)
    for s in range(n):
        dist = {s: 0}
        stack = [s]
        while stack:
            u = stack.pop()
            for v in adj[u]:
                if v not in dist:
                    dist[v] = dist[u] + 1
                    stack.append(v)
        r = np.linalg.norm(lig.xyz - lig.xyz[s], axis=1)
        for j in range(n):
            if dist[j] == 2:
                assert r[j] >= 1.2 - 1e-4
            elif dist[j] >= 3:
                assert r[j] >= min_nonlocal - 1e-4
    assert abs(float(np.sum(lig.charges, dtype=np.float64))) < 1e-4
    assert np.allclose(lig.xyz.mean(axis=0), 0.0, atol=1e-4)


@pytest.mark.parametrize("n,t", [(1, 0), (2, 0), (3, 1), (24, 5), (60, 15), (100, 32)])
def test_python_ligand_is_valid(n, t):
    lig = synth.ligand(n * 7 + t, n, t)
    check_ligand(lig)
    assert lig.n_torsions <= t


def test_fast_ligand_set_is_valid_and_seeded():
    L = synth.ligand_set_fast(3, 300)
    for lig in L[:120]:
        check_ligand(lig)
    n = np.array([l.n_atoms for l in L])
    assert n.min() >= 10 and n.max() <= 100 and 25 <= np.median(n) <= 40
    again = synth.ligand_set_fast(3, 5)
    for a, b in zip(L, again):
        assert np.array_equal(a.xyz, b.xyz) and np.array_equal(a.types, b.types)
    other = synth.ligand_set_fast(4, 5)
    assert not all(np.array_equal(a.types, b.types) for a, b in zip(L, other))


def test_packed_ligand_set_matches_the_list():
    L = synth.ligand_set_fast(6, 400)
    P = synth.ligand_set_fast(6, 400, packed=True)
    assert len(P) == 400 and P.n_atoms_per_ligand.sum() == len(P.types) == len(P.xyz)
    assert P.n_bonds_per_ligand.sum() == len(P.bonds) == len(P.rotatable)
    for i in (0, 1, 199, 399):
        a, b = L[i], P[i]
        assert np.array_equal(a.types, b.types) and np.array_equal(a.xyz, b.xyz)
        assert np.array_equal(a.charges, b.charges) and np.array_equal(a.bonds, b.bonds)
        assert np.array_equal(a.rotatable, b.rotatable)
    S = P.subset([7, 3])
    assert np.array_equal(S[0].xyz, L[7].xyz) and np.array_equal(S[1].bonds, L[3].bonds)
    R = synth.pack_ligands(L[:50])
    assert np.array_equal(R.xyz, P.xyz[:R.n_atoms_per_ligand.sum()])


def test_fast_ligand_type_frequencies():
    L = synth.ligand_set_fast(9, 2000, atoms=(20, 40), dist="uniform")
    t = np.concatenate([l.types for l in L])
    f = np.bincount(t, minlength=len(synth.TYPE_TABLE)) / len(t)
    for name, p in synth.FREQ_SIX.items():
        # HD that finds no host becomes C, so allow a small shift between the two
        assert abs(f[synth.TYPE_ID[name]] - p) < (0.02 if name in ("C", "HD") else 0.01), name


def test_screen_helpers():
    from paper_2007_03678_amd import screen
    judge = np.array([5.0, -3.0, 0.0, -9.0, 2.0, -1.0, 7.0, -4.0, 1.0, 3.0])
    assert list(screen.top_fraction(judge, 0.2)) == [3, 7]
    assert len(screen.top_fraction(judge, 0.25)) == 3
    assert screen.recall(judge, [7, 3, 0], top_frac=0.2) == (2, 2)
    assert screen.recall(judge, [7, 0], top_frac=0.2) == (1, 2)
    # a perfect predictor needs exactly the top fraction; a reversed one needs all
    assert screen.fraction_for_recall(judge, judge, 1.0, 0.2) == pytest.approx(0.2)
    assert screen.fraction_for_recall(-judge, judge, 1.0, 0.2) == pytest.approx(1.0)
    assert screen.fraction_for_recall(-judge, judge, 0.5, 0.2) == pytest.approx(0.9)
    lo, hi = screen.clopper_pearson(19, 20)
    assert lo == pytest.approx(0.7513, abs=1e-3) and hi == pytest.approx(0.9987, abs=1e-3)
    assert screen.clopper_pearson(0, 10)[0] == 0.0 and screen.clopper_pearson(10, 10)[1] == 1.0


def test_size_prior_helpers():
    from scipy.stats import rankdata
    from paper_2007_03678_amd import screen
    rng = np.random.default_rng(3)
    n = 400
    nat = rng.integers(10, 100, n).astype(float)
    pred = rng.normal(size=n)
    assert np.array_equal(screen.prior_score(pred, nat, 0.0), rankdata(pred))
    s = screen.prior_score(pred, nat, 1.0)
    assert np.array_equal(s, rankdata(pred) + rankdata(-nat))
    # ties share the mean of their ranks
    assert screen.average_rank([3.0, 1.0, 3.0, 2.0, 3.0]).tolist() == [4.0, 1.0, 4.0, 2.0, 4.0]
    heavy = rng.integers(0, 5, 1000).astype(float)
    assert np.array_equal(screen.average_rank(heavy), rankdata(heavy))
    # labels that reward size beyond what the prediction knows: a positive weight wins
    labels = -nat + 5.0 * rng.normal(size=n)
    w, f = screen.choose_prior_weight(pred, labels, nat, top_frac=0.05)
    assert w > 0 and f <= screen.fraction_for_recall(pred, labels, 0.95, 0.05)
    # a perfect prediction needs no prior
    w0, f0 = screen.choose_prior_weight(labels, labels, nat, top_frac=0.05)
    assert w0 == 0.0 and f0 == pytest.approx(19 / 400)   # 19 of the 20 positives first
