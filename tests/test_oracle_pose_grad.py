"""Pins for the oracle's ligand preparation, pose and analytic gradient (CPU).

Pose: a hand-derived 4-atom case, rigid-fragment and bond-length
preservation, identity genotype, 2*pi periodicity, and agreement of the
deepest-first and root-first torsion orders.  Gradient: central finite
differences of the energy in every degree of freedom, zero net force and
torque of the intramolecular part, and the a cos + b sin + c shape of a
single torsion under an affine field.
"""
import math
import os

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
T = synth.TYPE_ID


def chain4():
    xyz = np.array([[-0.5, 1, 0], [0, 0, 0], [1.5, 0, 0], [2, 1, 0]], np.float32)
    return synth.Ligand(np.array([T["C"]] * 4, np.int32), np.zeros(4, np.float32), xyz,
                        np.array([[0, 1], [1, 2], [2, 3]], np.int32), np.array([0, 1, 0], np.uint8))


def test_hand_derived_four_atom_pose(orc):
    L = orc.ligand(chain4())
    assert L.root_atom == 1 and L.n_tor == 1 and L.n_pairs == 0
    a, b, depth, moves = L.torsion(0)
    assert (a, b, depth) == (1, 2, 1) and moves.tolist() == [False, False, True, True]
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "pose_4atom.txt"))
            if l.strip() and not l.startswith("#")]
    c = np.array([0.75, 0.5, 0.0])
    for r in rows:
        v = [float(x) for x in r]
        g = np.zeros(40)
        g[0:3] = c
        g[3:7] = v[1:5]
        g[7] = v[0]
        xyz = orc.pose(L, g)
        assert np.allclose(xyz[3], v[5:8], atol=1e-12)


def test_pair_set_of_a_chain(orc):
    xyz = np.array([[0, 0, 0], [1.5, 0, 0], [2, 1.4, 0], [3.5, 1.4, 0], [4, 2.8, 0], [5.5, 2.8, 0]], np.float32)
    bonds = np.array([[0, 1], [1, 2], [2, 3], [3, 4], [4, 5]], np.int32)
    for rot in ([0, 0, 1, 0, 0], [0, 1, 1, 0, 0]):
        lig = synth.Ligand(np.array([T["C"]] * 6, np.int32), np.zeros(6, np.float32), xyz, bonds,
                           np.array(rot, np.uint8))
        assert sorted(orc.ligand(lig).pairs()) == [(0, 4), (0, 5), (1, 5)]
    # no rotatable bond: one rigid body, no pairs
    lig = synth.Ligand(np.array([T["C"]] * 6, np.int32), np.zeros(6, np.float32), xyz, bonds,
                       np.zeros(5, np.uint8))
    assert orc.ligand(lig).pairs() == []


@pytest.mark.parametrize("case", ["cycle", "disconnected", "terminal", "index", "selfloop", "toolarge",
                                  "toomanytor"])
def test_ligand_validation(orc, case):
    lig = synth.ligand(1, 10, 2)
    b, r, n = lig.bonds.copy(), lig.rotatable.copy(), lig.n_atoms
    types, q, xyz = lig.types, lig.charges, lig.xyz
    if case == "cycle":
        b[0] = [b[1][0], b[1][1]]
    elif case == "disconnected":
        b = b[:-1]
        r = r[:-1]
    elif case == "terminal":
        leaf = [i for i in range(n) if np.sum(b == i) == 1][0]
        k = int(np.where((b == leaf).any(axis=1))[0][0])
        r[k] = 1
    elif case == "index":
        b[2] = [0, n]
    elif case == "selfloop":
        b[2] = [3, 3]
    elif case == "toolarge":
        big = synth.ligand(2, 128, 3)
        types = np.concatenate([big.types, [0]]).astype(np.int32)
        q = np.concatenate([big.charges, [0]]).astype(np.float32)
        xyz = np.concatenate([big.xyz, [[9, 9, 9]]]).astype(np.float32)
        b = np.concatenate([big.bonds, [[0, 128]]]).astype(np.int32)
        r = np.concatenate([big.rotatable, [0]]).astype(np.uint8)
    elif case == "toomanytor":
        big = synth.ligand(3, 100, 40)
        types, q, xyz, b = big.types, big.charges, big.xyz, big.bonds
        deg = np.bincount(b.ravel(), minlength=100)
        r = ((deg[b[:, 0]] >= 2) & (deg[b[:, 1]] >= 2)).astype(np.uint8)
        assert r.sum() > 32
    with pytest.raises(ValueError):
        orc.ligand(synth.Ligand(types, q, xyz, b, r))


def bond_lengths(lig, xyz):
    return np.linalg.norm(xyz[lig.bonds[:, 0]] - xyz[lig.bonds[:, 1]], axis=1)


@pytest.mark.parametrize("seed,n,t", [(1, 24, 5), (2, 60, 15), (3, 100, 32), (4, 12, 0)])
def test_pose_preserves_geometry(orc, seed, n, t):
    lig = synth.ligand(seed, n, t, shuffle=True)
    L = orc.ligand(lig)
    grid = synth.make_grid(40, 0.375)
    ref = lig.xyz.astype(np.float64)
    c = ref.mean(axis=0)
    ident = np.zeros(40)
    ident[0:3] = c
    ident[3] = 1.0
    assert np.allclose(orc.pose(L, ident), ref, atol=1e-12)
    frag = fragments(lig)
    for g in synth.random_genotypes(seed, 8, L.n_tor, grid):
        x0 = orc.pose(L, g.astype(np.float64), order=0)
        x1 = orc.pose(L, g.astype(np.float64), order=1)
        assert np.allclose(x0, x1, atol=1e-10)
        assert np.allclose(bond_lengths(lig, x0), bond_lengths(lig, ref), atol=1e-12)
        g2 = g.astype(np.float64).copy()
        g2[7:7 + L.n_tor] += 2 * math.pi
        assert np.allclose(orc.pose(L, g2), x0, atol=1e-10)
        # atoms of one rigid fragment keep all their distances
        for f in set(frag):
            idx = [i for i in range(n) if frag[i] == f]
            d0 = np.linalg.norm(ref[idx][:, None] - ref[idx][None], axis=2)
            d1 = np.linalg.norm(x0[idx][:, None] - x0[idx][None], axis=2)
            assert np.allclose(d0, d1, atol=1e-11)


def fragments(lig):
    """Components of the bond graph without its rotatable bonds."""
    parent = list(range(lig.n_atoms))

    def find(i):
        while parent[i] != i:
            i = parent[i]
        return i
    for (a, b), r in zip(lig.bonds, lig.rotatable):
        if not r:
            parent[find(int(a))] = find(int(b))
    return [find(i) for i in range(lig.n_atoms)]


def test_permutation_invariance(orc):
    """Relabelled atoms and reordered / flipped bonds describe the same molecule:
    the same energy once torsion angles follow their bonds."""
    rec = synth.receptor(5, 300, side=12.0)
    grid = synth.make_grid(16, 0.375, map_types=synth.SIX_TYPES)
    G = orc.grid(grid, rec)
    lig = synth.ligand(21, 30, 7)
    rng = np.random.default_rng(4)
    ap, bp = rng.permutation(lig.n_atoms), rng.permutation(len(lig.bonds))
    lig2 = synth.permute(lig, ap, bp, rng)
    L1, L2 = orc.ligand(lig), orc.ligand(lig2)
    rot1 = np.where(lig.rotatable)[0]               # bond index of torsion k
    rot2 = np.where(lig2.rotatable)[0]
    # torsion k of lig2 is bond rot2[k] of lig2 = bond bp[rot2[k]] of lig
    tmap = [int(np.where(rot1 == bp[b])[0][0]) for b in rot2]
    for g in synth.random_genotypes(2, 5, L1.n_tor, grid, margin=2.0):
        g = g.astype(np.float64)
        g2 = g.copy()
        g2[7:7 + L1.n_tor] = g[7 + np.array(tmap)] if L1.n_tor else []
        assert orc.score(L2, G, g2)[0] == pytest.approx(orc.score(L1, G, g)[0], rel=1e-10)


def qmul(a, b):
    return np.array([a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3],
                     a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2],
                     a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1],
                     a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0]])


def rotvec_quat(w):
    th = np.linalg.norm(w)
    if th == 0:
        return np.array([1.0, 0, 0, 0])
    return np.concatenate([[math.cos(th / 2)], math.sin(th / 2) * w / th])


def fd_gradient(orc, L, G, g, h=1e-5):
    """Central differences: t directly, omega via q <- exp(w/2) q, theta directly."""
    out = np.zeros(40)
    qn = g[3:7] / np.linalg.norm(g[3:7])
    for d in range(3):
        gp, gm = g.copy(), g.copy()
        gp[d] += h
        gm[d] -= h
        out[d] = (orc.score(L, G, gp)[0] - orc.score(L, G, gm)[0]) / (2 * h)
    for d in range(3):
        w = np.zeros(3)
        w[d] = h
        gp, gm = g.copy(), g.copy()
        gp[3:7] = qmul(rotvec_quat(w), qn)
        gm[3:7] = qmul(rotvec_quat(-w), qn)
        out[3 + d] = (orc.score(L, G, gp)[0] - orc.score(L, G, gm)[0]) / (2 * h)
    for k in range(L.n_tor):
        gp, gm = g.copy(), g.copy()
        gp[7 + k] += h
        gm[7 + k] -= h
        out[7 + k] = (orc.score(L, G, gp)[0] - orc.score(L, G, gm)[0]) / (2 * h)
    return out


def away_from_faces(xyz, grid, margin):
    u = (xyz - np.array(grid.origin)) / grid.spacing
    f = u - np.floor(u)
    inside = np.all((u > 0) & (u < np.array(grid.n) - 1))
    return inside and np.all((f > margin) & (f < 1 - margin))


@pytest.mark.parametrize("seed,n,t", [(31, 20, 4), (32, 40, 10), (33, 70, 20)])
def test_gradient_matches_central_differences(orc, seed, n, t):
    rec = synth.receptor(seed, 500, side=16.0)
    grid = synth.make_grid(30, 0.375, map_types=synth.SIX_TYPES)
    G = orc.grid(grid, rec)
    lig = synth.ligand(seed, n, t)
    L = orc.ligand(lig)
    checked = 0
    for g in synth.random_genotypes(seed, 60, L.n_tor, grid, margin=3.0):
        g = g.astype(np.float64)
        E, grad, _, xyz = orc.score(L, G, g, want_xyz=True)
        # the interpolant is only C0 across cell faces: skip poses with an atom
        # closer to a face than the largest finite-difference displacement
        if not away_from_faces(xyz, grid, 2e-3):
            continue
        fd = fd_gradient(orc, L, G, g, h=1e-5)
        scale = max(np.linalg.norm(grad), 1.0)
        assert np.linalg.norm(fd - grad) <= 1e-6 * scale, (fd - grad)[:7 + L.n_tor]
        checked += 1
        if checked == 3:
            break
    assert checked >= 1


def test_intramolecular_force_and_torque_vanish(orc):
    """With all maps zero the energy is intramolecular only: the net force and
    torque on the ligand are zero (the pair forces act along the pair axis)."""
    grid = synth.make_grid(60, 0.5, map_types=synth.SIX_TYPES)
    G = orc.grid(grid, values=np.zeros((8, 60, 60, 60), np.float32))
    lig = synth.ligand(41, 45, 12)
    L = orc.ligand(lig)
    for g in synth.random_genotypes(1, 6, L.n_tor, grid, margin=12.0):
        E, grad, terms = orc.score(L, G, g.astype(np.float64))
        assert terms[0] == 0.0
        scale = np.abs(grad[7:7 + L.n_tor]).max() + 1.0
        assert np.abs(grad[0:6]).max() <= 1e-9 * scale


def test_single_torsion_is_harmonic_in_affine_field(orc):
    """A 4-atom chain has no intramolecular pair; in an affine field the energy
    as a function of its one torsion is a cos(theta) + b sin(theta) + c."""
    grid = synth.make_grid(20, 0.5, map_types=[T["C"]])
    rng = np.random.default_rng(2)
    coef = [(0.3, rng.normal(size=3)), (0.0, np.zeros(3)), (0.0, np.zeros(3))]
    nx = 20
    z, y, x = np.meshgrid(np.arange(nx), np.arange(nx), np.arange(nx), indexing="ij")
    P = [grid.origin[0] + 0.5 * x, grid.origin[1] + 0.5 * y, grid.origin[2] + 0.5 * z]
    vals = np.stack([a + b[0] * P[0] + b[1] * P[1] + b[2] * P[2] for a, b in coef]).astype(np.float32)
    G = orc.grid(grid, values=vals)
    L = orc.ligand(chain4())
    g = np.zeros(40)
    g[0:3] = grid.center
    g[3:7] = [0.9, 0.1, -0.3, 0.2]

    def E(th):
        gg = g.copy()
        gg[7] = th
        return orc.score(L, G, gg)[0]
    c0, cp, cq = E(0.0), E(math.pi), E(math.pi / 2)
    c = 0.5 * (c0 + cp)
    a = c0 - c
    b = cq - c
    for th in rng.uniform(-math.pi, math.pi, 10):
        assert E(th) == pytest.approx(a * math.cos(th) + b * math.sin(th) + c, abs=1e-5)
