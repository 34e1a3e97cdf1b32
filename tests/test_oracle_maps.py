"""Pins for the oracle's grid maps and trilinear interpolation (CPU only).

Maps are pinned to the pair potentials (themselves pinned by closed forms):
a ligand atom at a node scores exactly its direct pair sum with the
receptor.  Interpolation is pinned by exactness on affine fields, node
values, superposition, lattice symmetry and the out-of-grid restraint.
"""
import math

import numpy as np
import pytest

import synth

T = synth.TYPE_ID


def one_atom_ligand(t, q):
    return synth.Ligand(np.array([t], np.int32), np.array([q], np.float32), np.zeros((1, 3), np.float32),
                        np.zeros((0, 2), np.int32), np.zeros(0, np.uint8))


def geno_at(x, n_tor=0):
    g = np.zeros(40)
    g[0:3] = x
    g[3] = 1.0
    return g


def test_node_value_is_pair_sum_with_receptor(orc, ff):
    """Atom at a node: map_t + q map_e + |q| map_d == sum_a pair(t, q; a), with the
    vdW / H-bond / desolvation part limited to the cutoff."""
    rec = synth.receptor(3, 300, side=12.0)
    grid = synth.make_grid(12, 0.375, map_types=synth.ALL_TYPES)
    G = orc.grid(grid, rec)
    rng = np.random.default_rng(0)
    for _ in range(12):
        i, j, k = rng.integers(0, 12, size=3)
        p = np.array(grid.origin) + grid.spacing * np.array([i, j, k])
        exact = G.node_exact(int(i), int(j), int(k))
        for t in (T["C"], T["OA"], T["HD"], T["SA"]):
            q = float(np.float32(rng.normal(0, 0.3)))
            ref = 0.0
            for a in range(len(rec.types)):
                r = float(np.linalg.norm(p - rec.xyz[a].astype(np.float64)))
                ta, qa = int(rec.types[a]), float(rec.charges[a])
                if r < ff["cutoff"]:
                    ref += orc.pair(t, q, ta, qa, r)[0]
                else:
                    ref += orc.elec(q, qa, r)[0]
            m = grid.map_types.index(t)
            val = exact[m] + q * exact[-2] + abs(q) * exact[-1]
            if exact[m] < ff["cap"]:
                assert val == pytest.approx(ref, rel=1e-10, abs=1e-10)


def test_single_receptor_atom_radial_profile(orc, ff):
    """One receptor atom at a node: values along an axis follow the pair terms
    of the distance, identical in the six axis directions."""
    grid = synth.make_grid(21, 0.375, map_types=[T["C"], T["HD"]])
    c = np.array(grid.origin) + 10 * grid.spacing
    rec = synth.Receptor(c[None].astype(np.float32), np.array([T["OA"]], np.int32),
                         np.array([-0.4], np.float32))
    G = orc.grid(grid, rec)
    v = G.values()
    for s in range(1, 11):
        r = s * grid.spacing
        ref_c = orc.lj(T["C"], T["OA"], r)[0] + orc.desolv(T["C"], 0.0, T["OA"], -0.4, r)[0]
        ref_hd = orc.lj(T["HD"], T["OA"], r)[0] + orc.desolv(T["HD"], 0.0, T["OA"], -0.4, r)[0]
        ref_e = orc.elec(1.0, -0.4, r)[0]
        for (i, j, k) in ((10 + s, 10, 10), (10 - s, 10, 10), (10, 10 + s, 10), (10, 10 - s, 10),
                          (10, 10, 10 + s), (10, 10, 10 - s)):
            assert v[0, k, j, i] == pytest.approx(min(ref_c, ff["cap"]), rel=1e-6)
            assert v[1, k, j, i] == pytest.approx(min(ref_hd, ff["cap"]), rel=1e-6)
            assert v[2, k, j, i] == pytest.approx(ref_e, rel=1e-6)
    # at the atom itself the affinity maps hit the cap
    assert v[0, 10, 10, 10] == ff["cap"] and v[1, 10, 10, 10] == ff["cap"]


def test_superposition_of_receptors(orc):
    rA = synth.receptor(1, 80, side=10.0)
    rB = synth.receptor(2, 70, side=10.0)
    rAB = synth.Receptor(np.concatenate([rA.xyz, rB.xyz]), np.concatenate([rA.types, rB.types]),
                         np.concatenate([rA.charges, rB.charges]))
    grid = synth.make_grid(8, 0.5, map_types=synth.SIX_TYPES)
    GA, GB, GAB = orc.grid(grid, rA), orc.grid(grid, rB), orc.grid(grid, rAB)
    for (i, j, k) in ((0, 0, 0), (3, 4, 5), (7, 7, 7), (1, 6, 2)):
        a, b, ab = GA.node_exact(i, j, k), GB.node_exact(i, j, k), GAB.node_exact(i, j, k)
        ok = ab[:-2] < 1e5
        assert np.allclose((a + b)[:-2][ok], ab[:-2][ok], rtol=1e-12, atol=1e-12)
        assert np.allclose((a + b)[-2:], ab[-2:], rtol=1e-12, atol=1e-14)


def test_lazy_grid_equals_full_grid(orc):
    rec = synth.receptor(4, 200, side=10.0)
    grid = synth.make_grid(10, 0.4, map_types=synth.SIX_TYPES)
    full = orc.grid(grid, rec).values()
    lazy = orc.grid(grid, rec, lazy=True)
    for (i, j, k) in ((0, 0, 0), (9, 2, 5), (4, 4, 4)):
        assert np.array_equal(lazy.node(i, j, k), full[:, k, j, i])


def affine_maps(grid, coef):
    """Map m = a_m + b_m . p at every node (coef: [(a, b[3]), ...] for all maps)."""
    nx, ny, nz = grid.n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    P = [grid.origin[0] + grid.spacing * x, grid.origin[1] + grid.spacing * y, grid.origin[2] + grid.spacing * z]
    return np.stack([a + b[0] * P[0] + b[1] * P[1] + b[2] * P[2] for a, b in coef]).astype(np.float64)


def test_trilinear_exact_on_affine_fields(orc):
    grid = synth.make_grid((9, 11, 13), 0.5, center=(1.0, -2.0, 0.5), map_types=[T["C"], T["OA"]])
    rng = np.random.default_rng(5)
    coef = [(rng.normal(), rng.normal(size=3)) for _ in range(4)]
    vals = affine_maps(grid, coef).astype(np.float32)
    G = orc.grid(grid, values=vals)
    lo, hi = np.array(grid.origin), np.array(grid.origin) + np.array(grid.extent)
    for _ in range(40):
        x = rng.uniform(lo + 0.01, hi - 0.01)
        for t, m in ((T["C"], 0), (T["OA"], 1)):
            q = float(rng.normal(0, 0.3))
            L = orc.ligand(one_atom_ligand(t, q))
            E, g, _ = orc.score(L, G, geno_at(x))
            # fp32-stored affine maps: compare with the stored node values' field
            b = coef[m][1] + np.float32(q) * coef[2][1] + abs(np.float32(q)) * coef[3][1]
            a = coef[m][0] + np.float32(q) * coef[2][0] + abs(np.float32(q)) * coef[3][0]
            assert E == pytest.approx(a + b @ x, abs=2e-5 * (1 + abs(a) + np.abs(b).sum() * 10))
            assert np.allclose(g[0:3], b, atol=1e-4 * (1 + np.abs(b).max()))


def test_atom_on_node_gets_node_value_and_restraint_outside(orc, ff):
    grid = synth.make_grid(6, 0.375, map_types=[T["N"]])
    rng = np.random.default_rng(9)
    vals = rng.normal(size=(3, 6, 6, 6)).astype(np.float32)
    G = orc.grid(grid, values=vals)
    q = float(np.float32(-0.27))   # ligand charges are float32 inputs
    L = orc.ligand(one_atom_ligand(T["N"], q))
    for (i, j, k) in ((0, 0, 0), (5, 5, 5), (2, 3, 4), (5, 0, 3)):
        x = np.array(grid.origin) + grid.spacing * np.array([i, j, k])
        E, _, _ = orc.score(L, G, geno_at(x))
        ref = float(vals[0, k, j, i]) + q * float(vals[1, k, j, i]) + abs(q) * float(vals[2, k, j, i])
        assert E == pytest.approx(ref, rel=1e-12, abs=1e-12)
    # 0.7 A beyond the +x face at node (5,2,1): value of that face node + k_out d^2, gradient 2 k_out d
    x = np.array(grid.origin) + grid.spacing * np.array([5, 2, 1]) + np.array([0.7, 0, 0])
    E, g, _ = orc.score(L, G, geno_at(x))
    node = float(vals[0, 1, 2, 5]) + q * float(vals[1, 1, 2, 5]) + abs(q) * float(vals[2, 1, 2, 5])
    assert E == pytest.approx(node + ff["k_out"] * 0.49, rel=1e-12)
    assert g[0] == pytest.approx(2 * ff["k_out"] * 0.7, rel=1e-12)


def test_lattice_rotation_invariance(orc):
    """Rotate ligand and maps together by 90 degrees about z through the grid
    centre: the energy is unchanged."""
    rec = synth.receptor(6, 400, side=12.0)
    grid = synth.make_grid(16, 0.375, map_types=synth.SIX_TYPES)
    vals = orc.grid(grid, rec).values()
    # rotation about +z by 90 deg: new(x,y) = (-y, x) about the centre.  A node (i,j) of the
    # rotated field takes the value of the original node (j, n-1-i).
    rot = np.empty_like(vals)
    n = 16
    for i in range(n):
        for j in range(n):
            rot[:, :, j, i] = vals[:, :, n - 1 - i, j]
    G0 = orc.grid(grid, values=vals)
    G1 = orc.grid(grid, values=rot)
    c = np.array(grid.center)
    lig = synth.ligand(11, 18, 4)
    L = orc.ligand(lig)
    qz = np.array([math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4)])
    rng = np.random.default_rng(3)
    for g in synth.random_genotypes(8, 6, L.n_tor, grid, margin=2.0, normalize_q=True):
        g = g.astype(np.float64)
        E0, _, _ = orc.score(L, G0, g)
        g1 = g.copy()
        d = g[0:3] - c
        g1[0:3] = c + np.array([-d[1], d[0], d[2]])
        w, x, y, z = g[3:7]
        a = qz
        g1[3:7] = [a[0] * w - a[3] * z, a[0] * x - a[3] * y, a[0] * y + a[3] * x, a[0] * z + a[3] * w]
        E1, _, _ = orc.score(L, G1, g1)
        assert E1 == pytest.approx(E0, rel=1e-9, abs=1e-9)


def test_translation_invariance(orc):
    rec = synth.receptor(7, 300, side=12.0)
    grid = synth.make_grid(14, 0.375, map_types=synth.SIX_TYPES)
    vals = orc.grid(grid, rec).values()
    v = np.array([3.25, -1.5, 7.0])
    grid2 = synth.Grid(grid.n, grid.spacing, tuple(np.array(grid.origin) + v), grid.map_types)
    G0, G1 = orc.grid(grid, values=vals), orc.grid(grid2, values=vals)
    L = orc.ligand(synth.ligand(12, 15, 3))
    for g in synth.random_genotypes(9, 5, L.n_tor, grid, margin=1.5):
        g = g.astype(np.float64)
        g2 = g.copy()
        g2[0:3] += v
        assert orc.score(L, G1, g2)[0] == pytest.approx(orc.score(L, G0, g)[0], rel=1e-10, abs=1e-9)
